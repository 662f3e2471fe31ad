// Operator assembly kernels (setup only).
//
// The global operator A and every local operator A_j are the P1 discretisation
// of the complex-symmetric PML form (Section 1, eq. (pml)/(weak), multiplied
// through by gamma_1 gamma_2):
//     a(u,v) = int (g2/g1) u_x v_x + (g1/g2) u_y v_y - k^2 g1 g2 u v
// on right triangles (every cell cut along its SW-NE diagonal), coefficients
// at the triangle centroids.  With that cut the stiffness couples only the
// four axis neighbours; the mass adds the NE/SW diagonal.  A node's row is
// summed here from its six surrounding triangles (the closed-form 7-point
// stencil); triangles outside the assembly box are skipped, which gives the
// local operators on Omega_j (Section 2: a_j is a restricted to Omega_j, with
// the local stretch).  Local impedance (Section 3 (ii)) adds
// -i k gamma_t (h/6)[2 1; 1 2] on every edge of Gamma_j.
#include "device.h"

namespace raspml {

namespace {

struct Stretch {
    bool lo, hi;
    double a, b;
};

struct Coef {
    cplx<double> cx, cy, cm;
};

__device__ __forceinline__ cplx<double> cdiv(cplx<double> a, cplx<double> b) {
    return cmul(a, crecip(b));
}

__device__ __forceinline__ Coef tri_coef(const DevProb &P, int ci, int cj, bool lower,
                                         const Stretch &sx, const Stretch &sy) {
    const double h = P.h;
    const double x = (ci - P.G) * h + (lower ? 2.0 * h / 3.0 : h / 3.0);
    const double y = (cj - P.G) * h + (lower ? h / 3.0 : 2.0 * h / 3.0);
    cplx<double> g1 = gamma_at(x, P.sigma, sx.lo, sx.a, sx.hi, sx.b);
    cplx<double> g2 = gamma_at(y, P.sigma, sy.lo, sy.a, sy.hi, sy.b);
    return {cdiv(g2, g1), cdiv(g1, g2), cmul(g1, g2)};
}

// Row of node (i, j): out[0] diagonal, out[1] coupling to (i+1, j),
// out[2] to (i, j+1), out[3] to (i+1, j+1).  Cells (ci, cj) with
// bx0 <= ci < bx1 and by0 <= cj < by1 contribute.
__device__ void row_entries(const DevProb &P, int i, int j, int bx0, int bx1, int by0, int by1,
                            const Stretch &sx, const Stretch &sy, int imp, cplx<double> out[4]) {
    const double h = P.h, k2 = P.k * P.k;
    auto in = [&](int ci, int cj) { return ci >= bx0 && ci < bx1 && cj >= by0 && cj < by1; };
    cplx<double> KC{0, 0}, KE{0, 0}, KN{0, 0}, MC{0, 0}, ME{0, 0}, MN{0, 0}, MNE{0, 0};
    if (in(i, j)) {                       // L_ij (node = SW corner), U_ij (SW corner)
        Coef L = tri_coef(P, i, j, true, sx, sy);
        Coef U = tri_coef(P, i, j, false, sx, sy);
        KC = cadd(KC, cadd(L.cx, U.cy));
        KE = cadd(KE, L.cx);
        KN = cadd(KN, U.cy);
        MC = cadd(MC, cadd(L.cm, U.cm));
        ME = cadd(ME, L.cm);
        MN = cadd(MN, U.cm);
        MNE = cadd(L.cm, U.cm);
    }
    if (in(i, j - 1)) {                   // U_{i,j-1} (node = NW corner)
        Coef U = tri_coef(P, i, j - 1, false, sx, sy);
        KC = cadd(KC, cadd(U.cx, U.cy));
        KE = cadd(KE, U.cx);
        MC = cadd(MC, U.cm);
        ME = cadd(ME, U.cm);
    }
    if (in(i - 1, j)) {                   // L_{i-1,j} (node = SE corner)
        Coef L = tri_coef(P, i - 1, j, true, sx, sy);
        KC = cadd(KC, cadd(L.cx, L.cy));
        KN = cadd(KN, L.cy);
        MC = cadd(MC, L.cm);
        MN = cadd(MN, L.cm);
    }
    if (in(i - 1, j - 1)) {               // L and U of cell (i-1, j-1) (node = NE corner)
        Coef L = tri_coef(P, i - 1, j - 1, true, sx, sy);
        Coef U = tri_coef(P, i - 1, j - 1, false, sx, sy);
        KC = cadd(KC, cadd(L.cy, U.cx));
        MC = cadd(MC, cadd(L.cm, U.cm));
    }
    const double m6 = h * h / 12.0, m12 = h * h / 24.0;
    out[0] = csub(cscale(KC, 0.5), cscale(MC, k2 * m6));
    out[1] = csub(cscale(KE, -0.5), cscale(ME, k2 * m12));
    out[2] = csub(cscale(KN, -0.5), cscale(MN, k2 * m12));
    out[3] = cscale(MNE, -k2 * m12);

    if (imp == 0) return;
    // impedance: -i k gamma_t (h/3) on the diagonal, (h/6) off the diagonal
    const cplx<double> mik{0.0, -P.k};
    auto edge_y = [&](int jj) {          // edge (x, jj)-(x, jj+1): tangential stretch in y
        double ym = (jj - P.G) * h + 0.5 * h;
        return cmul(mik, gamma_at(ym, P.sigma, sy.lo, sy.a, sy.hi, sy.b));
    };
    auto edge_x = [&](int ii) {
        double xm = (ii - P.G) * h + 0.5 * h;
        return cmul(mik, gamma_at(xm, P.sigma, sx.lo, sx.a, sx.hi, sx.b));
    };
    const bool on_x = ((imp & SD_IMP_XLO) && i == bx0) || ((imp & SD_IMP_XHI) && i == bx1);
    const bool on_y = ((imp & SD_IMP_YLO) && j == by0) || ((imp & SD_IMP_YHI) && j == by1);
    if (on_x) {
        if (j >= by0 && j < by1) {
            cplx<double> g = edge_y(j);
            out[0] = cadd(out[0], cscale(g, h / 3.0));
            out[2] = cadd(out[2], cscale(g, h / 6.0));
        }
        if (j - 1 >= by0 && j - 1 < by1) out[0] = cadd(out[0], cscale(edge_y(j - 1), h / 3.0));
    }
    if (on_y) {
        if (i >= bx0 && i < bx1) {
            cplx<double> g = edge_x(i);
            out[0] = cadd(out[0], cscale(g, h / 3.0));
            out[1] = cadd(out[1], cscale(g, h / 6.0));
        }
        if (i - 1 >= bx0 && i - 1 < bx1) out[0] = cadd(out[0], cscale(edge_x(i - 1), h / 3.0));
    }
}

__global__ void k_global_stencil(const DevProb *__restrict__ probs, double2 *__restrict__ coef,
                                 long long ntot) {
    const DevProb P = probs[blockIdx.y];
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const int i = static_cast<int>(idx % P.n1) + 1;
    const int j = static_cast<int>(idx / P.n1) + 1;
    Stretch none{false, false, 0.0, 0.0};
    cplx<double> r[4];
    row_entries(P, i, j, 0, P.Nc, 0, P.Nc, none, none, 0, r);
    if (i == P.n1) r[1] = {0, 0};
    if (j == P.n1) r[2] = {0, 0};
    if (i == P.n1 || j == P.n1) r[3] = {0, 0};
    const long long g = P.dof_off + idx;
    for (int e = 0; e < 4; ++e) coef[e * ntot + g] = make_double2(r[e].re, r[e].im);
}

__global__ void k_local_stencil(const DevProb *__restrict__ probs, const DevSub *__restrict__ subs,
                                double2 *__restrict__ lst) {
    const DevSub S = subs[blockIdx.y];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= S.n) return;
    const DevProb P = probs[S.prob];
    int i, j;
    if (S.xfast) {
        i = S.ix0 + r % S.nx;
        j = S.jy0 + r / S.nx;
    } else {
        j = S.jy0 + r % S.ny;
        i = S.ix0 + r / S.ny;
    }
    Stretch sx{(S.flags & SD_PML_XLO) != 0, (S.flags & SD_PML_XHI) != 0, S.ax, S.bx};
    Stretch sy{(S.flags & SD_PML_YLO) != 0, (S.flags & SD_PML_YHI) != 0, S.ay, S.by};
    const int imp = S.flags & (SD_IMP_XLO | SD_IMP_XHI | SD_IMP_YLO | SD_IMP_YHI);
    cplx<double> e[4];
    row_entries(P, i, j, S.bx0, S.bx1, S.by0, S.by1, sx, sy, imp, e);
    const int ix1 = S.ix0 + S.nx - 1, jy1 = S.jy0 + S.ny - 1;
    const bool okx = i + 1 <= ix1, oky = j + 1 <= jy1;
    if (!okx) e[1] = {0, 0};
    if (!oky) e[2] = {0, 0};
    if (!(okx && oky)) e[3] = {0, 0};
    cplx<double> fast = S.xfast ? e[1] : e[2];
    cplx<double> slow = S.xfast ? e[2] : e[1];
    double2 *o = lst + 4 * (S.loc_off + r);
    o[0] = make_double2(e[0].re, e[0].im);
    o[1] = make_double2(fast.re, fast.im);
    o[2] = make_double2(slow.re, slow.im);
    o[3] = make_double2(e[3].re, e[3].im);
}

// b = M f with the unweighted P1 mass matrix: h^2/2 on the diagonal and
// h^2/12 to the E, W, N, S, NE and SW neighbours.
__global__ void k_rhs(const DevProb *__restrict__ probs, const double2 *__restrict__ f,
                      double2 *__restrict__ b) {
    const DevProb P = probs[blockIdx.y];
    const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= P.ndof) return;
    const int n1 = P.n1;
    const int i = static_cast<int>(idx % n1) + 1;
    const int j = static_cast<int>(idx / n1) + 1;
    const double2 *F = f + P.dof_off;
    auto at = [&](int ii, int jj) {
        if (ii < 1 || ii > n1 || jj < 1 || jj > n1) return make_double2(0.0, 0.0);
        return F[static_cast<long long>(jj - 1) * n1 + (ii - 1)];
    };
    double2 c = at(i, j);
    double sr = 0.0, si = 0.0;
    const int di[6] = {1, -1, 0, 0, 1, -1};
    const int dj[6] = {0, 0, 1, -1, 1, -1};
    for (int t = 0; t < 6; ++t) {
        double2 v = at(i + di[t], j + dj[t]);
        sr += v.x;
        si += v.y;
    }
    const double h2 = P.h * P.h;
    b[P.dof_off + idx] = make_double2(h2 / 2.0 * c.x + h2 / 12.0 * sr, h2 / 2.0 * c.y + h2 / 12.0 * si);
}

}  // namespace

void launch_global_stencil(const DevProb *probs, int nprob, long long max_ndof, double2 *coef,
                           long long ntot, hipStream_t st) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    hipLaunchKernelGGL(k_global_stencil, grid, dim3(256), 0, st, probs, coef, ntot);
}

void launch_local_stencil(const DevProb *probs, const DevSub *subs, int nsub, int max_n,
                          double2 *lst, hipStream_t st) {
    dim3 grid(static_cast<unsigned>((max_n + 255) / 256), nsub);
    hipLaunchKernelGGL(k_local_stencil, grid, dim3(256), 0, st, probs, subs, lst);
}

void launch_rhs(const DevProb *probs, int nprob, long long max_ndof, const double2 *f,
                double2 *b, hipStream_t st) {
    dim3 grid(static_cast<unsigned>((max_ndof + 255) / 256), nprob);
    hipLaunchKernelGGL(k_rhs, grid, dim3(256), 0, st, probs, f, b);
}

}  // namespace raspml
