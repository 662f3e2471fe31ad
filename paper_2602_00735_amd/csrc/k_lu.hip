// Batched band factorisation A_j = L_j D_j L_j^T without pivoting (setup).
//
// The paper does not name its local solver; its setup/solve split (Table 4)
// is read as one factorisation of every local operator, reused by every
// preconditioner application.  A_j is complex symmetric (A_j = A_j^T), so its
// no-pivot LU is U = D L^T: L (twice, by columns and by rows) and D^{-1}
// are stored, never U.
//
// One workgroup factorises one subdomain.  The active (W x W) window of the
// band, W = half-bandwidth + 1, lives in registers as a ring: band row r sits
// in slot r mod W, so the window slides one position per column without
// moving data.  Thread (ty, tx) owns the slots {ty + TY a} x {tx + TX b}.
// Per column c:
//   1. the owners of column slot c mod W publish column c to LDS;
//   2. every thread forms l = column / pivot and applies the rank-1 update
//      S -= l u^T to its slots;
//   3. L[:, c] is written in slot order (row r at position r mod W, the
//      pivot position holds 0), D^{-1}_c separately, and every entry L[r, c]
//      also into row r of a second, row-ordered copy R (position c mod W) so
//      that the backward sweep can run in column form too.  R holds its rows
//      last row first: the backward sweep then reads it front to back, and the
//      two sweeps together read one contiguous stream [L | R];
//   4. the retired slot receives the band row/column c + W, whose only
//      non-zeros are the 7-point stencil couplings (diagonal, fast -1,
//      slow -n_fast, diagonal -n_fast-1), staged in LDS one block of 64 rows
//      ahead.  (W may exceed the band by one slot: it is rounded up to even
//      for the solve; that slot stays zero.)
// One barrier per column (the column buffer is double buffered).  Rows past
// the matrix end (padding to a multiple of 64) are identity rows.
#include "device.h"

namespace raspml {

namespace {

template <typename T>
struct Eps;
template <>
struct Eps<float> {
    static constexpr float tol = 1e-6f;
};
template <>
struct Eps<double> {
    static constexpr double tol = 1e-14;
};

// Stencil value entering the window: entry e (0: diagonal, 1: coupling to
// r-1, 2: to r-nf, 3: to r-nf-1) of band row r.
template <typename T>
__device__ __forceinline__ cplx<T> incoming(const double2 *__restrict__ lst, int n, int nf,
                                            int r, int e) {
    if (r >= n) return cplx<T>{e == 0 ? T(1) : T(0), T(0)};
    double2 v = make_double2(0.0, 0.0);
    const bool wrap = (r % nf) == 0;        // r starts a new fast line
    if (e == 0)
        v = lst[4 * static_cast<long long>(r) + 0];
    else if (e == 1 && !wrap && r >= 1)
        v = lst[4 * static_cast<long long>(r - 1) + 1];
    else if (e == 2 && r >= nf)
        v = lst[4 * static_cast<long long>(r - nf) + 2];
    else if (e == 3 && !wrap && r >= nf + 1)
        v = lst[4 * static_cast<long long>(r - nf - 1) + 3];
    return cplx<T>{static_cast<T>(v.x), static_cast<T>(v.y)};
}

// A_j(r, c) for r, c inside the first window (r, c < W).
template <typename T>
__device__ __forceinline__ cplx<T> initial_entry(const double2 *__restrict__ lst, int n, int nf,
                                                 int r, int c) {
    if (r < c) {
        int t = r;
        r = c;
        c = t;
    }
    const int d = r - c;
    if (r >= n) return cplx<T>{d == 0 ? T(1) : T(0), T(0)};
    cplx<T> v{0, 0};
    if (d == 0) v = cadd(v, incoming<T>(lst, n, nf, r, 0));
    if (d == 1) v = cadd(v, incoming<T>(lst, n, nf, r, 1));
    if (d == nf) v = cadd(v, incoming<T>(lst, n, nf, r, 2));
    if (d == nf + 1) v = cadd(v, incoming<T>(lst, n, nf, r, 3));
    return v;
}

template <typename T, int TY, int TX, int RY, int RX>
__global__ __launch_bounds__(TY *TX) void k_band_ldlt(const DevSub *__restrict__ subs,
                                                      const int *__restrict__ order,
                                                      const double2 *__restrict__ lst_all,
                                                      cplx<T> *__restrict__ F,
                                                      int *__restrict__ status) {
    constexpr int MW = TY * RY;
    static_assert(TX * RX == MW, "square window");
    constexpr int NT = TY * TX;
    __shared__ cplx<T> ubuf[2][MW];
    __shared__ cplx<T> newrow[2][64][4];
    __shared__ T dorig[MW];

    const int s = order[blockIdx.x];
    const DevSub S = subs[s];
    const int W = S.W, nf = S.nf, n = S.n, npad = S.npad;
    const int tid = threadIdx.x;
    const int ty = tid / TX, tx = tid % TX;
    const double2 *lst = lst_all + 4 * S.loc_off;
    cplx<T> *L = F + S.fac_off;
    cplx<T> *Rw = L + static_cast<long long>(npad) * W;        // rows of L, last first
    cplx<T> *Dinv = Rw + static_cast<long long>(npad) * W;

    cplx<T> A[RY][RX];
#pragma unroll
    for (int a = 0; a < RY; ++a)
#pragma unroll
        for (int b = 0; b < RX; ++b) {
            const int rs = ty + TY * a, cs = tx + TX * b;
            A[a][b] = (rs < W && cs < W) ? initial_entry<T>(lst, n, nf, rs, cs) : cplx<T>{0, 0};
        }
    for (int i = tid; i < 2 * MW; i += NT) ubuf[i / MW][i % MW] = cplx<T>{0, 0};
    // Row r < W of R has no columns before 0 at positions r+1 .. W-1; every
    // other entry of L, R and D^{-1} is written by the column loop below.
    for (int i = tid; i < W * W; i += NT) {
        const int r = i / W, q = i % W;
        if (q > r && r < npad) Rw[static_cast<long long>(npad - 1 - r) * W + q] = cplx<T>{0, 0};
    }
    for (int i = tid; i < W; i += NT) {
        cplx<T> d = initial_entry<T>(lst, n, nf, i, i);
        dorig[i] = sqrt(cabs2(d));
    }
    cplx<T> nxt{0, 0};
    if (tid < 256) {
        newrow[0][tid >> 2][tid & 3] = incoming<T>(lst, n, nf, W + (tid >> 2), tid & 3);
        nxt = incoming<T>(lst, n, nf, W + 64 + (tid >> 2), tid & 3);
    }
    int bad = -1;
    __syncthreads();

    int sl = 0;
    for (int c = 0; c < npad; ++c) {
        const int buf = c & 1;
        if ((c & 63) == 0 && c > 0) {
            if (tid < 256) {
                newrow[(c >> 6) & 1][tid >> 2][tid & 3] = nxt;
                nxt = incoming<T>(lst, n, nf, W + c + 64 + (tid >> 2), tid & 3);
            }
        }
        // 1. publish column c (owners of column slot sl)
        if (tx == sl % TX) {
            const int bsel = sl / TX;
#pragma unroll
            for (int b = 0; b < RX; ++b)
                if (b == bsel)
#pragma unroll
                    for (int a = 0; a < RY; ++a) {
                        const int rs = ty + TY * a;
                        if (rs < W) ubuf[buf][rs] = A[a][b];
                    }
        }
        __syncthreads();
        const cplx<T> piv = ubuf[buf][sl];
        const cplx<T> dinv = crecip(piv);
        if (tid == 0) {
            const T ap = sqrt(cabs2(piv));
            if (bad < 0 && !(ap > Eps<T>::tol * dorig[sl] && ap < T(1e30))) bad = c;
        }
        // 2. rank-1 update of the window
        cplx<T> u[RX], l[RY];
#pragma unroll
        for (int b = 0; b < RX; ++b) u[b] = ubuf[buf][tx + TX * b];
#pragma unroll
        for (int a = 0; a < RY; ++a) l[a] = cmul(ubuf[buf][ty + TY * a], dinv);
#pragma unroll
        for (int a = 0; a < RY; ++a)
#pragma unroll
            for (int b = 0; b < RX; ++b) A[a][b] = cfms(A[a][b], l[a], u[b]);
        // 3. write L[:, c] in slot order, each entry also into its row of R,
        //    and D^{-1}_c; slot p holds row c + ((p - sl) mod W)
        for (int p = tid; p < W; p += NT) {
            const cplx<T> lv = (p == sl) ? cplx<T>{0, 0} : cmul(ubuf[buf][p], dinv);
            L[static_cast<long long>(c) * W + p] = lv;
            const int r = c + (p >= sl ? p - sl : p - sl + W);
            if (r < npad) Rw[static_cast<long long>(npad - 1 - r) * W + sl] = lv;
        }
        if (tid == 0) Dinv[c] = dinv;
        // 4. band row/column c + W enters slot sl
        const cplx<T> *nr = newrow[(c >> 6) & 1][c & 63];
        const cplx<T> eC = nr[0], eE = nr[1], eN = nr[2], eNE = nr[3];
        // slots of rows c+W-1, c+W-nf and c+W-nf-1 (W - nf is 2, or 3 when W
        // was rounded up to even)
        const int sm1 = sl == 0 ? W - 1 : sl - 1;
        const int sp1 = sl + 1 == W ? 0 : sl + 1;
        const int sN = sl + (W - nf) >= W ? sl + (W - nf) - W : sl + (W - nf);
        const int sNE = sN == 0 ? W - 1 : sN - 1;
        auto value = [&](int q) {
            cplx<T> v{0, 0};
            if (q == sl) v = cadd(v, eC);
            if (q == sm1) v = cadd(v, eE);
            if (q == sN) v = cadd(v, eN);
            if (q == sNE) v = cadd(v, eNE);
            return v;
        };
        if (ty == sl % TY) {
            const int asel = sl / TY;
#pragma unroll
            for (int a = 0; a < RY; ++a)
                if (a == asel)
#pragma unroll
                    for (int b = 0; b < RX; ++b) A[a][b] = value(tx + TX * b);
        }
        if (tx == sl % TX) {
            const int bsel = sl / TX;
#pragma unroll
            for (int b = 0; b < RX; ++b)
                if (b == bsel)
#pragma unroll
                    for (int a = 0; a < RY; ++a) A[a][b] = value(ty + TY * a);
        }
        if (tid == 0) dorig[sl] = sqrt(cabs2(eC));
        sl = sp1;
    }
    if (tid == 0) status[s] = bad;
}

template <typename T, int TY, int TX, int RY, int RX>
void launch_cfg(const DevSub *subs, const int *order, int nsub, const double2 *lst, void *F,
                int *status, hipStream_t st) {
    hipLaunchKernelGGL((k_band_ldlt<T, TY, TX, RY, RX>), dim3(nsub), dim3(TY * TX), 0, st, subs,
                       order, lst, static_cast<cplx<T> *>(F), status);
}

}  // namespace

// maxW: largest W of the batch (<= kMaxW).
void launch_band_ldlt(bool fp64, int maxW, const DevSub *subs, const int *order, int nsub,
                      const double2 *lst, void *F, int *status, hipStream_t st) {
    if (fp64) {
        if (maxW <= 64)
            launch_cfg<double, 16, 16, 4, 4>(subs, order, nsub, lst, F, status, st);
        else if (maxW <= 96)
            launch_cfg<double, 16, 16, 6, 6>(subs, order, nsub, lst, F, status, st);
        else
            launch_cfg<double, 16, 32, 8, 4>(subs, order, nsub, lst, F, status, st);
    } else {
        if (maxW <= 64)
            launch_cfg<float, 16, 16, 4, 4>(subs, order, nsub, lst, F, status, st);
        else if (maxW <= 96)
            launch_cfg<float, 16, 16, 6, 6>(subs, order, nsub, lst, F, status, st);
        else
            launch_cfg<float, 16, 32, 8, 4>(subs, order, nsub, lst, F, status, st);
    }
}

}  // namespace raspml
