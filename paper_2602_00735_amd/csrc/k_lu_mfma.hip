// Blocked band factorisation A_j = L_j D_j L_j^T (complex64 or complex128,
// no pivoting) with the trailing update on the matrix cores (setup).
//
// Same factor as the one-column kernel (Section 2's local solves; A_j is
// complex symmetric, U = D L^T), organised in panels of 16 columns:
//   1. the panel (16 columns of the active window) is factorised in
//      registers: for each column, the pivot is broadcast with v_readlane,
//      the column is scaled, and the panel's later columns take the rank-1
//      update;
//   2. L, its row copy and D^{-1} of the 16 columns are written out;
//   3. the rest of the window takes the rank-16 update C -= L W^T with
//      W = L D, as complex 16x16 tiles: 16 v_mfma_f32_16x16x4f32 (complex64)
//      or v_mfma_f64_16x16x4f64 (complex128) per tile (real and imaginary
//      parts in four real products).  Only tiles on or below the diagonal
//      are updated: the window stays symmetric.
// The window covers M = 16 NT rows and columns, NT = ceil((W + 15) / 16),
// enough to hold every row a panel column reaches (W - 1 below its
// diagonal).  Its NT (NT + 1) / 2 tiles on and below the diagonal live in
// the accumulator registers, spread over the four waves.  Tile (I, J) lies
// on tile diagonal d = I - J; the tiles of one diagonal form a ring of
// length NT - d, so when the window slides by one panel no tile moves: each
// diagonal's ring index advances, and the tile that leaves (J = 0) becomes
// that diagonal's new last tile (J = NT - 1 - d, in the new last tile row),
// refilled from the stencil (those rows have not been touched by any earlier
// panel).  Rows past the matrix end are identity rows, as in the one-column
// kernel, and the factor layout is the same: columns of L in slot order,
// then the rows last row first, then D^{-1}.
//
// The panel factorisation runs on as few waves as hold its rows (two at
// M = 112): the column-by-column chain is serial, and every extra wave
// repeats it for the panel's first 16 rows; the other waves' issue slots
// stay free for the workgroups that share the CU.
#include "device.h"

namespace raspml {

namespace {

// Precision traits: the 16x16x4 matrix-core product, which takes
// A[l & 15][l >> 4] and B[l >> 4][l & 15] from lane l in both precisions and
// leaves D[row0(l) + rs r][l & 15] in accumulator r -- rows 4 (l >> 4) .. + 3
// in complex64 (v_mfma_f32_16x16x4f32), rows (l >> 4) + {0, 4, 8, 12} in
// complex128 (v_mfma_f64_16x16x4f64; measured lane by lane); the pivot
// reciprocal (v_rcp_f32 within 1 ulp for complex64 factors, v_rcp_f64 with
// two Newton steps for complex128) and the relative pivot test.
template <typename T>
struct Prec;
template <>
struct Prec<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // c + (-a) b
    static __device__ __forceinline__ v4 mfma_na(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(-a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ int row0(int lane) { return 4 * (lane >> 4); }
    static constexpr int rs = 1;
    static constexpr float tol = 1e-6f;
};
template <>
struct Prec<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // c + (-a) b: the f64 instruction's own negation of A (its last operand
    // is the neg:[a, b, c] modifier), no vector instruction for the sign
    static __device__ __forceinline__ v4 mfma_na(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
    }
    // v_rcp_f64 and two Newton steps r <- r + r (1 - x r): within an ulp or
    // two of 1/x (the division's scaling and fix-up steps, which make it
    // correctly rounded and handle denormal and huge x, lie on the panel's
    // serial chain; |d|^2 of a pivot that passes the test is neither)
    static __device__ __forceinline__ double rcp(double x) {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        return fma(r, fma(-x, r, 1.0), r);
    }
    static __device__ __forceinline__ int row0(int lane) { return lane >> 4; }
    static constexpr int rs = 4;
    static constexpr double tol = 1e-14;
};

constexpr int kLdsStride = 17;   // complex values per LDS panel row (16 + 1 pad)

// Workgroup barrier for the LDS panel buffers only: waits for this wave's
// LDS accesses (lgkmcnt(0); vmcnt and expcnt left at their maximum), not for
// its global stores and loads (a fence would drain those, costing a memory
// round trip per barrier).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// A_j(r, q) from the local stencil: for r >= q the coupling is stored at
// node q, entry 0 (d = r - q = 0), 1 (d = 1), 2 (d = n_fast) or 3
// (d = n_fast + 1; entries 1 and 3 vanish when r starts a fast line).
// Identity past the matrix end.  Branch-free: one clamped load, always
// issued, so that its wait can sit at the first use of the value.
template <typename T>
__device__ __forceinline__ cplx<T> band_entry(const double2 *__restrict__ lst, int n, int nf,
                                              int r, int q) {
    const int hi = max(r, q), lo = min(r, q), d = hi - lo;
    const int e = d == 0 ? 0 : d == 1 ? 1 : d == nf ? 2 : 3;
    const bool wrap = (hi % nf) == 0;
    const bool in = hi < n;
    const bool coupled = in && (d == 0 || d == nf || ((d == 1 || d == nf + 1) && !wrap));
    const double2 v = lst[4LL * min(lo, n - 1) + e];
    const T id = (!in && d == 0) ? T(1) : T(0);
    return cplx<T>{coupled ? static_cast<T>(v.x) : id, coupled ? static_cast<T>(v.y) : T(0)};
}

// What one panel needs from the stencil, staged in LDS a panel ahead so that
// no global load waits inside the panel: entries i < 64 are the couplings of
// row r = c0 + M + i / 4 (the rows entering the window's last tile row) to
// rows r - {0, 1, n_fast, n_fast + 1} (i mod 4), entries 64..79 the
// magnitudes |A_j(c, c)| of the panel's columns c = c0 + i - 64 (pivot
// test).  stage_load issues the one load of entry i, stage_value finishes it
// where the value is written to LDS.
struct StageRef {
    int r, q;        // entry A_j(r, q), r >= q
    bool diag;       // magnitude of a diagonal entry
};
__device__ __forceinline__ StageRef stage_ref(int i, int c0, int M, int nf) {
    if (i < 64) {
        const int r = c0 + M + (i >> 2), e = i & 3;
        return {r, r - (e == 0 ? 0 : e == 1 ? 1 : e == 2 ? nf : nf + 1), false};
    }
    const int c = c0 + i - 64;
    return {c, c, true};
}
__device__ __forceinline__ double2 stage_load(const double2 *__restrict__ lst, int n, int nf,
                                              const StageRef &a) {
    const int d = a.r - a.q;
    const int e = d == 0 ? 0 : d == 1 ? 1 : d == nf ? 2 : 3;
    return lst[4LL * min(a.q, n - 1) + e];
}
template <typename T>
__device__ __forceinline__ cplx<T> stage_value(int n, int nf, const StageRef &a, double2 v) {
    const int d = a.r - a.q;
    const bool wrap = (a.r % nf) == 0;
    const bool in = a.r < n;
    const bool coupled = in && (d == 0 || d == nf || ((d == 1 || d == nf + 1) && !wrap));
    const T id = (!in && d == 0) ? T(1) : T(0);
    const cplx<T> x{coupled ? static_cast<T>(v.x) : id, coupled ? static_cast<T>(v.y) : T(0)};
    return a.diag ? cplx<T>{sqrt(cabs2(x)), T(0)} : x;
}

// Rows of the panel factorisation: NW = 1 + ceil((M - 64) / 48) waves take
// part.  Part v = 0 holds rows 0..63 (one per lane); part v >= 1 holds rows
// 0..15 in lanes 0..15 (the same values as part 0, computed again so that no
// wave waits for another) and rows 64 + 48 (v - 1) + lane - 16 in lanes 16..63.
template <int M>
constexpr int panel_waves() { return M <= 64 ? 1 : 1 + (M - 64 + 47) / 48; }

// Panel factorisation on the calling wave's rows.  Before column k is
// scaled, its entries below the diagonal are L[row, k] d_k, i.e. W = L D,
// which is what the later panel columns need (the values of rows j < 16,
// broadcast with v_readlane) and what is stored in WB; L goes to LP, except
// for the first 16 rows, whose L goes to LT (every part reads those rows of
// LP first).  Entries on and above the diagonal are not zeroed: no reader
// uses them.  dg: lane k < 16 holds
// |A_j(c0 + k, c0 + k)| for the pivot test.  The reciprocal of the pivot is
// Prec<T>::rcp of |d|^2.
template <typename T, int M>
__device__ __forceinline__ int factor_panel(cplx<T> *LP, cplx<T> *LT, cplx<T> *WB, T dg, int c0,
                                            cplx<T> *__restrict__ Dinv, int bad, int part) {
    const int lane = threadIdx.x & 63;
    const int row = part == 0 ? lane : lane < 16 ? lane : 64 + 48 * (part - 1) + lane - 16;
    const bool have = row < M;
    const cplx<T> zero{T(0), T(0)};
    cplx<T> x[16];
    const cplx<T> *src = LP + min(row, M - 1) * kLdsStride;
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = csel(have, src[k], zero);
    // lanes with nothing to store write the spare row M of LP / WB
    cplx<T> *dl = lane < 16 ? (part == 0 ? LT + row * kLdsStride : LP + M * kLdsStride)
                            : LP + min(row, M) * kLdsStride;
    cplx<T> *dw = WB + (lane < 16 ? M : min(row, M)) * kLdsStride;
    T pa = T(0);                    // lane k: |d_k|^2, tested after the loop
    cplx<T> dinv = zero;            // lane k: 1 / d_k
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const cplx<T> w = x[k];                          // W[row, k] for row > k
        const cplx<T> d = readlane(w, k);
        const T m2 = cabs2(d);
        pa = writelane(pa, m2, k);
        const T rm = Prec<T>::rcp(m2);
        const cplx<T> inv{d.re * rm, -d.im * rm};
        dinv = writelane(dinv, inv, k);
        const cplx<T> l = cmul(w, inv);
#pragma unroll
        for (int j = k + 1; j < 16; ++j) x[j] = cfms(x[j], l, readlane(w, j));
        // (rows k and above hold values no reader uses: the column and row
        // copies read L strictly below the diagonal, the update rows >= 16)
        dl[k] = l;
        dw[k] = w;
    }
    if (part == 0 && lane < 16) Dinv[c0 + lane] = dinv;
    const T ad = sqrt(pa);
    const bool fail = lane < 16 && !(ad > Prec<T>::tol * dg && ad < T(1e30));
    const unsigned long long fm = __ballot(fail);
    if (bad < 0 && fm != 0) bad = c0 + __builtin_ctzll(fm);
    return bad;
}

// Lower tile number u < NT (NT + 1) / 2 as (diagonal d, ring slot q); the
// loop is bounded, so numbers past the last tile give d = NT (unused).
template <int NT>
__device__ __forceinline__ void lower_tile(int u, int &d, int &q) {
    d = 0;
    int left = u;
#pragma unroll
    for (int dd = 0; dd < NT; ++dd) {
        if (d == dd && left >= NT - dd) {
            left -= NT - dd;
            d = dd + 1;
        }
    }
    q = left;
}

// OCC: the kernel is held to the register budget of four workgroups per CU
// (complex64: 128 registers; at k = 640 all 1024 subdomains are then
// resident at once; from NT = 6 on the window spills a little to fit) or of
// two (complex128: 256 registers).  Without it the compiler's own budget
// applies (complex64: 146 registers at NT = 7, three workgroups per CU, no
// spills).  Which is faster depends on the window and the number of
// subdomains; the autotuner measures both.
template <typename T, int NT, bool OCC>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(OCC ? (sizeof(T) == 4 ? 4 : 2) : 1))) void
k_band_ldlt_mfma(const DevSub *__restrict__ subs, const int *__restrict__ order,
                 const double2 *__restrict__ lst_all, cplx<T> *__restrict__ F,
                 int *__restrict__ status) {
    typedef typename Prec<T>::v4 v4;
    constexpr int M = 16 * NT;
    constexpr int NL = NT * (NT + 1) / 2;   // tiles on and below the diagonal
    constexpr int NS = (NL + 3) / 4;        // tile slots per wave
    static_assert(panel_waves<M>() <= 4, "panel rows per wave");
    // row M of LP and WB is a spare row for lanes with nothing to store
    __shared__ cplx<T> LP[(M + 1) * kLdsStride];   // published panel, then L (rows 16..)
    __shared__ cplx<T> LT[16 * kLdsStride];        // L of the panel's first 16 rows
    __shared__ cplx<T> WB[(M + 1) * kLdsStride];   // W = L D (rows 16..)
    __shared__ cplx<T> STG[2][80];                 // stencil staged per panel parity

    const int sid = order[blockIdx.x];
    const DevSub S = subs[sid];
    const int W = S.W, nf = S.nf, n = S.n, npad = S.npad;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fwave = blockIdx.x & 3;
    const int part = (wave - fwave) & 3;   // panel part of this wave
    const double2 *lst = lst_all + 4 * S.loc_off;
    cplx<T> *L = F + S.fac_off;
    cplx<T> *Rw = L + static_cast<long long>(npad) * W;   // rows of L, last first
    cplx<T> *Dinv = Rw + static_cast<long long>(npad) * W;
    // accumulator r of a tile holds its element (ti + RS r, tj)
    constexpr int RS = Prec<T>::rs;
    const int ti = Prec<T>::row0(lane), tj = lane & 15;
    const cplx<T> zero{T(0), T(0)};

    // Row r < W of R has no columns before 0 at positions r+1 .. W-1.
    for (int i = tid; i < W * W; i += 256) {
        const int r = i / W, q = i % W;
        if (q > r && r < npad) Rw[static_cast<long long>(npad - 1 - r) * W + q] = zero;
    }

    // slot s of this wave holds lower tile u = 4 s + wave: diagonal d, ring
    // slot q; at panel p its logical column is J = (q - p) mod (NT - d) and
    // its row I = J + d.  Window at panel 0: rows 16 I.., columns 16 J..
    v4 cre[NS], cim[NS];
    int dg_[NS], jc_[NS];            // diagonal and current logical column of each slot
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int d, q;
        lower_tile<NT>(4 * s + wave, d, q);
        const bool valid = 4 * s + wave < NL;
        dg_[s] = valid ? d : -1;
        jc_[s] = q;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cplx<T> v =
                valid ? band_entry<T>(lst, n, nf, 16 * (q + d) + ti + RS * r, 16 * q + tj) : zero;
            cre[s][r] = v.re;
            cim[s][r] = v.im;
        }
    }

    int bad = -1;
    // staged entries of panel 0; every thread loads one (branch-free), the
    // first 80 store theirs
    const int si = min(tid, 79);
    {
        const StageRef a = stage_ref(si, 0, M, nf);
        const cplx<T> v = stage_value<T>(n, nf, a, stage_load(lst, n, nf, a));
        if (tid < 80) STG[0][tid] = v;
    }
    lds_barrier();
    for (int c0 = 0; c0 < npad; c0 += 16) {
        const int buf = (c0 >> 4) & 1;
        // the next panel's entries: loaded now, stored at the end of the panel
        const double2 rnext = stage_load(lst, n, nf, stage_ref(si, c0 + 16, M, nf));
        const T dg = STG[buf][64 + tj].re;
        // 1. publish logical tile column 0 (J == 0 on every diagonal)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (dg_[s] >= 0 && jc_[s] == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    LP[(16 * dg_[s] + ti + RS * r) * kLdsStride + tj] = cplx<T>{cre[s][r], cim[s][r]};
            }
        }
        lds_barrier();
        // 2. panel factorisation
        // parts 0 .. NW-1 on waves fwave, fwave+1, ... (mod 4): the choice
        // rotates with the workgroup so that the workgroups sharing a CU
        // tend to factorise on different SIMDs
        if (part < panel_waves<M>()) bad = factor_panel<T, M>(LP, LT, WB, dg, c0, Dinv, bad, part);
        lds_barrier();
        // 3. columns c0 .. c0+15 of L (slot order) and their entries in the
        //    rows of L; row r's entry of column c sits at position c mod W
        {
            const int sl0 = c0 % W;
            const int pos = tid & 127;
#pragma unroll
            for (int k = tid >> 7; k < 16; k += 2) {
                const int c = c0 + k;
                int sl = sl0 + k;
                sl = sl >= W ? sl - W : sl;
                if (pos < W) {
                    const int r = c + (pos >= sl ? pos - sl : pos - sl + W);
                    const int rr = r - c0;
                    // one LDS read through a select of the two LDS arrays, the
                    // zero selected as a value (a select with a local would make a
                    // generic pointer and flat loads that wait on the stores)
                    const cplx<T> v = (rr < 16 ? LT : LP)[rr * kLdsStride + k];
                    L[static_cast<long long>(c) * W + pos] = csel(r == c, zero, v);
                }
            }
            const int k = tid & 15;
            int slk = sl0 + k;
            slk = slk >= W ? slk - W : slk;
            // row c's own position (c mod W) holds 0
            if (tid < 16) Rw[static_cast<long long>(npad - 1 - (c0 + k)) * W + slk] = zero;
            for (int r = c0 + 1 + (tid >> 4); r < c0 + W + 15; r += 16) {
                const int c = c0 + k;
                if (r > c && r < c + W && r < npad) {
                    const int rr = r - c0;
                    Rw[static_cast<long long>(npad - 1 - r) * W + slk] =
                        (rr < 16 ? LT : LP)[rr * kLdsStride + k];
                }
            }
        }
        // 4. rank-16 update of the tiles with J >= 1; the tiles with J == 0
        //    leave and come back as their diagonal's last tile
        int tdiff = ti - tj;
        asm volatile("" : "+v"(tdiff));   // per panel: keeps the per-slot offsets out of registers
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int d = dg_[s], J = jc_[s];
            if (d >= 0) {
                // the window slides: column J becomes J - 1, column 0 comes
                // back as the diagonal's last tile
                jc_[s] = J == 0 ? NT - 1 - d : J - 1;
                if (J >= 1) {
                    const int I = J + d;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int col = 4 * kk + (lane >> 4);
                        const cplx<T> l = LP[(16 * I + tj) * kLdsStride + col];
                        const cplx<T> w = WB[(16 * J + tj) * kLdsStride + col];
                        cre[s] = Prec<T>::mfma_na(l.re, w.re, cre[s]);
                        cre[s] = Prec<T>::mfma(l.im, w.im, cre[s]);
                        cim[s] = Prec<T>::mfma_na(l.re, w.im, cim[s]);
                        cim[s] = Prec<T>::mfma_na(l.im, w.re, cim[s]);
                    }
                } else {
                    // next window: row NT - 1, column NT - 1 - d, from the
                    // staged couplings of the entering rows; entry (ti + RS r,
                    // tj) of the tile lies dd = 16 d + ti + RS r - tj below the
                    // diagonal
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int dd = 16 * d + tdiff + RS * r;
                        const int e = dd == 0 ? 0 : dd == 1 ? 1 : dd == nf ? 2 : dd == nf + 1 ? 3 : -1;
                        const cplx<T> v = STG[buf][4 * (ti + RS * r) + max(e, 0)];
                        cre[s][r] = e >= 0 ? v.re : T(0);
                        cim[s][r] = e >= 0 ? v.im : T(0);
                    }
                }
            }
        }
        {
            const cplx<T> v = stage_value<T>(n, nf, stage_ref(si, c0 + 16, M, nf), rnext);
            if (tid < 80) STG[buf ^ 1][tid] = v;
        }
        lds_barrier();
    }
    if (part == 0 && lane == 0) status[sid] = bad;
}

template <typename T, int NT>
void launch_nt(bool occ, const DevSub *subs, const int *order, int count, const double2 *lst,
               void *F, int *status, hipStream_t st) {
    if (occ)
        hipLaunchKernelGGL((k_band_ldlt_mfma<T, NT, true>), dim3(count), dim3(256), 0, st, subs,
                           order, lst, static_cast<cplx<T> *>(F), status);
    else
        hipLaunchKernelGGL((k_band_ldlt_mfma<T, NT, false>), dim3(count), dim3(256), 0, st, subs,
                           order, lst, static_cast<cplx<T> *>(F), status);
}

template <typename T>
void launch_t(int NT, bool occ, const DevSub *subs, const int *order, int count,
              const double2 *lst, void *F, int *status, hipStream_t st) {
    switch (NT) {
        case 2: launch_nt<T, 2>(occ, subs, order, count, lst, F, status, st); break;
        case 3: launch_nt<T, 3>(occ, subs, order, count, lst, F, status, st); break;
        case 4: launch_nt<T, 4>(occ, subs, order, count, lst, F, status, st); break;
        case 5: launch_nt<T, 5>(occ, subs, order, count, lst, F, status, st); break;
        case 6: launch_nt<T, 6>(occ, subs, order, count, lst, F, status, st); break;
        case 7: launch_nt<T, 7>(occ, subs, order, count, lst, F, status, st); break;
        case 8: launch_nt<T, 8>(occ, subs, order, count, lst, F, status, st); break;
        default: launch_nt<T, 9>(occ, subs, order, count, lst, F, status, st); break;
    }
}

// ------------------------------------------------------------ wide bands
// W = 64 K with K = 3..7 (bands 129..447: the subdomains of Section 4's own
// experiments, 300-cell cores with their overlap and PML).  The same
// blocked LDL^T in 16-column panels, but the window (M = W + 16 rows and
// columns, NT = 4 K + 1 tiles per side, NT (NT + 1) / 2 tiles on and below
// the diagonal: 650 KB in complex64 at K = 6) no longer fits the register
// file: it lives in a global scratch of the workgroup's own (L2-resident),
// as the same diagonal rings.  Tile u of the scratch holds element
// (ti + RS r, tj) of lane l at u * 256 + 64 r + l, the matrix-core
// accumulator layout.  Per panel:
//   1. logical tile column 0 is read into LDS;
//   2. one wave factorises the 16 x 16 diagonal block (pivot broadcast with
//      v_readlane, as in the register kernel); every other row of the panel
//      is then one thread's 16-step forward substitution against it (the
//      pre-scaled block and the reciprocals from LDS);
//   3. L (column copy in slot order, row copy) and D^{-1} are written out,
//      in the layout of the other kernels with W the column length;
//   4. the tiles with J == 0 become their diagonal's entering tile,
//      straight from the stencil, and each wave takes its share of the tiles
//      with J >= 1 (C -= L_I (L_J D)^T on the matrix cores: loaded from the
//      scratch, 16 products, stored back), two at a time.
// The window at panel 0 holds the stencil's couplings; rows past the matrix
// end are identity rows.

// A_j(r, q) as band_entry, loading only where the stencil couples r and q.
template <typename T>
__device__ __forceinline__ cplx<T> band_entry_sparse(const double2 *__restrict__ lst, int n,
                                                     int nf, int r, int q) {
    const int hi = max(r, q), lo = min(r, q), d = hi - lo;
    const bool wrap = (hi % nf) == 0;
    const bool in = hi < n;
    const bool coupled = in && (d == 0 || d == nf || ((d == 1 || d == nf + 1) && !wrap));
    if (!coupled) return cplx<T>{(!in && d == 0) ? T(1) : T(0), T(0)};
    const int e = d == 0 ? 0 : d == 1 ? 1 : d == nf ? 2 : 3;
    const double2 v = lst[4LL * lo + e];
    return cplx<T>{static_cast<T>(v.x), static_cast<T>(v.y)};
}

// First tile of diagonal d in the rings (diagonal e has NT - e tiles).
template <int NT>
__device__ __forceinline__ int ring_base(int d) { return d * NT - d * (d - 1) / 2; }

// Threads per workgroup: as many waves as the registers allow (one
// workgroup per CU): twelve in complex64 (three per SIMD), eight in
// complex128.
template <typename T>
constexpr int wide_threads() { return sizeof(T) == 4 ? 768 : 512; }

template <typename T, int K>
__global__ __launch_bounds__(wide_threads<T>()) void k_band_ldlt_wide(
    const DevSub *__restrict__ subs, const int *__restrict__ order,
    const double2 *__restrict__ lst_all, cplx<T> *__restrict__ F, cplx<T> *__restrict__ scratch,
    int *__restrict__ status) {
    typedef typename Prec<T>::v4 v4;
    constexpr int W = 64 * K;
    constexpr int NT = 4 * K + 1;
    constexpr int M = 16 * NT;
    constexpr int NL = NT * (NT + 1) / 2;
    constexpr int NU = NT * (NT - 1) / 2;   // tiles a panel updates (J >= 1)
    constexpr int RS = Prec<T>::rs;
    constexpr int NTH = wide_threads<T>(), NWV = NTH / 64;
    __shared__ cplx<T> LP[M * kLdsStride];    // the panel; then L (zero on and above the diagonal)
    __shared__ cplx<T> WD[16 * kLdsStride];   // diagonal block, pre-scaled values (L D)
    __shared__ cplx<T> DV[16], IV[16];        // d_k and 1 / d_k of the panel's columns
    __shared__ int TQ[NL];                    // ring tile u: diagonal d (high half), slot q
    __shared__ int TU[NU];                    // update tile t: diagonal d (high half), column J

    const int sid = order[blockIdx.x];
    const DevSub S = subs[sid];
    const int nf = S.nf, n = S.n, npad = S.npad;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double2 *lst = lst_all + 4 * S.loc_off;
    cplx<T> *L = F + S.fac_off;
    cplx<T> *Rw = L + static_cast<long long>(npad) * W;   // rows of L, last first
    cplx<T> *Dinv = Rw + static_cast<long long>(npad) * W;
    cplx<T> *win = scratch + static_cast<long long>(blockIdx.x) * NL * 256;
    const int ti = Prec<T>::row0(lane), tj = lane & 15;
    const cplx<T> zero{T(0), T(0)};

    // Row r < W of R has no columns before 0 at positions r+1 .. W-1.
#pragma unroll 1
    for (int i = tid; i < W * W; i += NTH) {
        const int r = i / W, q = i % W;
        if (q > r && r < npad) Rw[static_cast<long long>(npad - 1 - r) * W + q] = zero;
    }
#pragma unroll 1
    for (int u = tid; u < NL; u += NTH) {
        int d = 0, q = u;
        while (q >= NT - d) q -= NT - d++;
        TQ[u] = (d << 16) | q;
    }
    // diagonal d has NT - 1 - d tiles with J >= 1
#pragma unroll 1
    for (int t = tid; t < NU; t += NTH) {
        int d = 0, j = t;
        while (j >= NT - 1 - d) j -= NT - 1 - d++;
        TU[t] = (d << 16) | (j + 1);
    }
    __syncthreads();
    // window at panel 0: ring tile (d, q) holds rows 16 (q + d).., columns 16 q..
#pragma unroll 1
    for (int u = wave; u < NL; u += NWV) {
        const int d = TQ[u] >> 16, q = TQ[u] & 0xffff;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            win[u * 256 + 64 * r + lane] =
                band_entry_sparse<T>(lst, n, nf, 16 * (q + d) + ti + RS * r, 16 * q + tj);
    }
    __syncthreads();

    int bad = -1;
#pragma unroll 1
    for (int c0 = 0; c0 < npad; c0 += 16) {
        const int p = c0 >> 4;
        // 1. logical tile column 0 (ring slot p mod (NT - I) of diagonal I)
#pragma unroll 1
        for (int I = wave; I < NT; I += NWV) {
            const cplx<T> *tile = win + (ring_base<NT>(I) + p % (NT - I)) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                LP[(16 * I + ti + RS * r) * kLdsStride + tj] = tile[64 * r + lane];
        }
        __syncthreads();
        // 2a. the diagonal block, rows 0..15 in lanes 0..15 of wave 0
        if (wave == 0) {
            const int row = min(lane, 15);
            cplx<T> x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = LP[row * kLdsStride + k];
            const int cd = c0 + row;            // |A_j(cd, cd)| for the pivot test
            const double2 a = lst[4LL * min(cd, n - 1)];
            const cplx<T> ad0{static_cast<T>(a.x), static_cast<T>(a.y)};
            const T dg = cd < n ? sqrt(cabs2(ad0)) : T(1);
            T pa = T(0);
            cplx<T> dinv = zero;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const cplx<T> w = x[k];
                const cplx<T> d = readlane(w, k);
                const T m2 = cabs2(d);
                pa = writelane(pa, m2, k);
                const T rm = Prec<T>::rcp(m2);
                const cplx<T> inv{d.re * rm, -d.im * rm};
                dinv = writelane(dinv, inv, k);
                const cplx<T> l = cmul(w, inv);
#pragma unroll
                for (int j = k + 1; j < 16; ++j) x[j] = cfms(x[j], l, readlane(w, j));
                if (lane < 16) {
                    LP[lane * kLdsStride + k] = csel(lane > k, l, zero);
                    WD[lane * kLdsStride + k] = w;
                }
                if (lane == k) {
                    DV[k] = d;
                    IV[k] = inv;
                }
            }
            if (lane < 16) Dinv[c0 + lane] = dinv;
            const T ad = sqrt(pa);
            const bool fail = lane < 16 && !(ad > Prec<T>::tol * dg && ad < T(1e30));
            const unsigned long long fm = __ballot(fail);
            if (bad < 0 && fm != 0) bad = c0 + __builtin_ctzll(fm);
        }
        __syncthreads();
        // 2b. rows 16 .. M-1 (the clobber keeps the block's LDS values from
        // being hoisted into registers across the at most two rows a thread
        // takes)
#pragma unroll 1
        for (int r = 16 + tid; r < M; r += NTH) {
            asm volatile("" ::: "memory");
            cplx<T> x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = LP[r * kLdsStride + k];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const cplx<T> l = cmul(x[k], IV[k]);
#pragma unroll
                for (int j = k + 1; j < 16; ++j) x[j] = cfms(x[j], l, WD[j * kLdsStride + k]);
                LP[r * kLdsStride + k] = l;
            }
        }
        __syncthreads();
        // 3. columns c0 .. c0+15 of L (slot order: row r at position r mod W,
        //    the column's own position 0) and their entries in the rows of L
        {
            const int sl0 = c0 % W;              // sl0 + 15 < W (W is a multiple of 64)
#pragma unroll 1
            for (int i = tid; i < 16 * W; i += NTH) {
                const int k = i / W, pos = i - (i / W) * W;
                const int c = c0 + k, sl = sl0 + k;
                const int r = c + (pos >= sl ? pos - sl : pos - sl + W);
                L[static_cast<long long>(c) * W + pos] =
                    r == c ? zero : LP[(r - c0) * kLdsStride + k];
            }
            const int k = tid & 15, c = c0 + k, slk = sl0 + k;
            if (tid < 16) Rw[static_cast<long long>(npad - 1 - c) * W + slk] = zero;
#pragma unroll 1
            for (int r = c0 + 1 + (tid >> 4); r < c0 + W + 15; r += NTH / 16)
                if (r > c && r < c + W && r < npad)
                    Rw[static_cast<long long>(npad - 1 - r) * W + slk] =
                        LP[(r - c0) * kLdsStride + k];
        }
        // 4. the tiles with J == 0 leave: their slots take their diagonal's
        //    entering tile (row NT - 1 of the next window), from the stencil
#pragma unroll 1
        for (int d = wave; d < NT; d += NWV) {
            cplx<T> *tile = win + (ring_base<NT>(d) + p % (NT - d)) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                tile[64 * r + lane] = band_entry_sparse<T>(
                    lst, n, nf, 16 * (p + NT) + ti + RS * r, 16 * (p + NT - d) + tj);
        }
        //    rank-16 update of the tiles with J >= 1 (logical (J + d, J),
        //    ring slot (p + J) mod (NT - d)), two per wave at a time so that
        //    the matrix-core chains of the two interleave; past the end the
        //    second repeats the last tile and is not stored
#pragma unroll 1
        for (int t = wave; t < NU; t += 2 * NWV) {
            const bool two = t + NWV < NU;
            const int tt[2] = {t, min(t + NWV, NU - 1)};
            int I[2], J[2];
            cplx<T> *tile[2];
            v4 cre[2], cim[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int d = TU[tt[h]] >> 16;
                J[h] = TU[tt[h]] & 0xffff;
                I[h] = J[h] + d;
                tile[h] = win + (ring_base<NT>(d) + (p + J[h]) % (NT - d)) * 256;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const cplx<T> v = tile[h][64 * r + lane];
                    cre[h][r] = v.re;
                    cim[h][r] = v.im;
                }
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int col = 4 * kk + (lane >> 4);
                const cplx<T> dv = DV[col];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const cplx<T> l = LP[(16 * I[h] + tj) * kLdsStride + col];
                    const cplx<T> w = cmul(LP[(16 * J[h] + tj) * kLdsStride + col], dv);
                    cre[h] = Prec<T>::mfma_na(l.re, w.re, cre[h]);
                    cim[h] = Prec<T>::mfma_na(l.re, w.im, cim[h]);
                    cre[h] = Prec<T>::mfma(l.im, w.im, cre[h]);
                    cim[h] = Prec<T>::mfma_na(l.im, w.re, cim[h]);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[0][64 * r + lane] = cplx<T>{cre[0][r], cim[0][r]};
            if (two) {
#pragma unroll
                for (int r = 0; r < 4; ++r) tile[1][64 * r + lane] = cplx<T>{cre[1][r], cim[1][r]};
            }
        }
        __syncthreads();
    }
    if (tid == 0) status[sid] = bad;
}

template <typename T>
void launch_wide_t(int K, const DevSub *subs, const int *order, int count, const double2 *lst,
                   void *F, void *scratch, int *status, hipStream_t st) {
    cplx<T> *Fc = static_cast<cplx<T> *>(F);
    cplx<T> *sc = static_cast<cplx<T> *>(scratch);
    const dim3 grid(count), block(wide_threads<T>());
#define RAS_WIDE(KK) \
    hipLaunchKernelGGL((k_band_ldlt_wide<T, KK>), grid, block, 0, st, subs, order, lst, Fc, sc, status)
    switch (K) {
        case 3: RAS_WIDE(3); break;
        case 4: RAS_WIDE(4); break;
        case 5: RAS_WIDE(5); break;
        case 6: RAS_WIDE(6); break;
        default: RAS_WIDE(7); break;
    }
#undef RAS_WIDE
}

}  // namespace

// Scratch elements (complex values) per workgroup of the wide factorisation
// for W = 64 K.
long long ldlt_wide_scratch(int K) {
    const long long NT = 4 * K + 1;
    return NT * (NT + 1) / 2 * 256;
}

// count subdomains order[0 .. count) that all have W == 64 K (K = 3..7);
// scratch: count * ldlt_wide_scratch(K) complex values of the factor
// precision.
void launch_band_ldlt_wide(bool fp64, int K, const DevSub *subs, const int *order, int count,
                           const double2 *lst, void *F, void *scratch, int *status,
                           hipStream_t st) {
    if (fp64)
        launch_wide_t<double>(K, subs, order, count, lst, F, scratch, status, st);
    else
        launch_wide_t<float>(K, subs, order, count, lst, F, scratch, status, st);
}

// Window tiles per side for a factor column length W (at most 128).
int ldlt_mfma_tiles(int W) { return (W + 15 + 15) / 16; }

// Default register budget of a window class (see k_band_ldlt_mfma).
bool ldlt_mfma_default_occ(bool fp64, int NT) { return fp64 ? true : NT <= 7; }

// count subdomains order[0 .. count) that all have ldlt_mfma_tiles(W) == NT.
void launch_band_ldlt_mfma(bool fp64, int NT, bool occ, const DevSub *subs, const int *order,
                           int count, const double2 *lst, void *F, int *status, hipStream_t st) {
    if (fp64)
        launch_t<double>(NT, occ, subs, order, count, lst, F, status, st);
    else
        launch_t<float>(NT, occ, subs, order, count, lst, F, status, st);
}

}  // namespace raspml
