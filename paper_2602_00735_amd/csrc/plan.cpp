// Host planner: parameter validation, Cartesian covering, subdomain PML
// extension and partition of unity (Section 2 "Cartesian covering" and
// partition of unity; Section 1 for the PML-extended square).
//
// Readings where the paper is silent (cell units throughout):
//   * Nc = grid + 2 G cells per side, node coordinates x_i = (i - G) h;
//     unknowns are the nodes 1..Nc-1 (Dirichlet on the boundary of Omega);
//   * cuts c_p = floor(p Nc / P); Omega_{p,int} = [c_p - delta, c_{p+1} + delta]
//     clipped to [0, Nc]; a PML of kappa cells is added on every side of
//     Omega_{p,int} that is not on the boundary of Omega; Omega_p is clipped
//     to [0, Nc];
//   * impedance: nodes on Gamma_j (boundary of Omega_j off the boundary of
//     Omega) are unknowns; Dirichlet: they are not;
//   * local numbering with the shorter side fastest, half-bandwidth
//     n_fast + 1;
//   * PoU: product of a left ramp (0 at c_p - delta, 1 at c_p + delta) and a
//     right ramp (1 at c_{p+1} - delta, 0 at c_{p+1} + delta), no ramp on a
//     side on the boundary of Omega, normalised to sum to one (Section 4:
//     tensor products of 1D functions linear across the overlaps); Boolean
//     variant: node i belongs to the chunk with c_p <= i < c_{p+1}.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "internal.h"

namespace raspml {

namespace {

struct Axis {
    int c_lo, c_hi, int_lo, int_hi, pml_lo, pml_hi, box_lo, box_hi, u_lo, u_hi;
    bool imp_lo, imp_hi;
};

Axis make_axis(int Nc, int P, int p, int delta, int kappa, int bc) {
    Axis a{};
    a.c_lo = static_cast<int>((static_cast<long long>(p) * Nc) / P);
    a.c_hi = static_cast<int>((static_cast<long long>(p + 1) * Nc) / P);
    a.int_lo = std::max(0, a.c_lo - delta);
    a.int_hi = std::min(Nc, a.c_hi + delta);
    a.pml_lo = a.int_lo > 0 ? kappa : 0;
    a.pml_hi = a.int_hi < Nc ? kappa : 0;
    a.box_lo = std::max(0, a.int_lo - a.pml_lo);
    a.box_hi = std::min(Nc, a.int_hi + a.pml_hi);
    if (bc == RAS_BC_IMP) {
        a.u_lo = std::max(a.box_lo, 1);
        a.u_hi = std::min(a.box_hi, Nc - 1);
        a.imp_lo = a.box_lo > 0;
        a.imp_hi = a.box_hi < Nc;
    } else {
        a.u_lo = a.box_lo + 1;
        a.u_hi = a.box_hi - 1;
        a.imp_lo = a.imp_hi = false;
    }
    return a;
}

double ramp_weight(const Axis &a, int Nc, int delta, int i) {
    double left = 1.0, right = 1.0;
    if (a.int_lo > 0) {
        if (delta > 0)
            left = std::min(1.0, std::max(0.0, (i - (a.c_lo - delta)) / (2.0 * delta)));
        else
            left = i >= a.c_lo ? 1.0 : 0.0;
    }
    if (a.int_hi < Nc) {
        if (delta > 0)
            right = std::min(1.0, std::max(0.0, ((a.c_hi + delta) - i) / (2.0 * delta)));
        else
            right = i <= a.c_hi ? 1.0 : 0.0;
    }
    return left * right;
}

// Fill the PoU table of one axis; returns false if a node has more than
// kMaxPou chunks with positive weight.
bool pou_axis(const std::vector<Axis> &ax, int Nc, int delta, int kind,
              std::vector<int> &cnt, std::vector<int> &chunk, std::vector<double> &w) {
    const int P = static_cast<int>(ax.size());
    cnt.assign(Nc + 1, 0);
    chunk.assign(static_cast<size_t>(Nc + 1) * kMaxPou, 0);
    w.assign(static_cast<size_t>(Nc + 1) * kMaxPou, 0.0);
    std::vector<double> raw(P);
    for (int i = 0; i <= Nc; ++i) {
        double s = 0.0;
        for (int p = 0; p < P; ++p) {
            double v;
            if (kind == RAS_POU_BOOLEAN)
                v = ((i >= ax[p].c_lo && i < ax[p].c_hi) || (p == P - 1 && i == Nc)) ? 1.0 : 0.0;
            else
                v = ramp_weight(ax[p], Nc, delta, i);
            raw[p] = v;
            s += v;
        }
        for (int p = 0; p < P; ++p) {
            if (raw[p] > 0.0) {
                if (cnt[i] == kMaxPou) return false;
                const size_t e = static_cast<size_t>(i) * kMaxPou + cnt[i];
                chunk[e] = p;
                w[e] = raw[p] / s;
                ++cnt[i];
            }
        }
    }
    return true;
}

bool bad(double x) { return !std::isfinite(x); }

}  // namespace

int plan_problem(double k, double h, const int grid[2], const int subdomains[2],
                 int overlap, int pml_width, const ras_pml_opts &opts,
                 PlanProblem &out, std::string &err) {
    char buf[256];
    if (bad(k) || k <= 0.0) { err = "k must be a positive finite number"; return RAS_EINVAL; }
    if (bad(h) || h <= 0.0) { err = "h must be a positive finite number"; return RAS_EINVAL; }
    if (grid == nullptr || subdomains == nullptr) { err = "grid/subdomains is NULL"; return RAS_EINVAL; }
    if (grid[0] < 1 || grid[1] != grid[0]) {
        err = "grid must be n x n cells with n >= 1 (the interior box is the unit square)";
        return RAS_EINVAL;
    }
    if (std::fabs(grid[0] * h - 1.0) > 1e-12) {
        std::snprintf(buf, sizeof buf, "grid * h = %.17g must equal 1", grid[0] * h);
        err = buf;
        return RAS_EINVAL;
    }
    // Section 3 (iii): a width argument of RAS_WIDTH_RULE takes the rule's value
    if (overlap == RAS_WIDTH_RULE) {
        const int rc = width_rule_cells(k, h, opts.width_c_delta, opts.width_k0, overlap, err);
        if (rc != RAS_OK) return rc;
    }
    if (pml_width == RAS_WIDTH_RULE) {
        const int rc = width_rule_cells(k, h, opts.width_c_kappa, opts.width_k0, pml_width, err);
        if (rc != RAS_OK) return rc;
    }
    if (overlap < 0 || pml_width < 0) {
        err = "overlap and pml_width must be >= 0 (or RAS_WIDTH_RULE)";
        return RAS_EINVAL;
    }
    if (opts.bc != RAS_BC_IMP && opts.bc != RAS_BC_DRCH) { err = "unknown bc"; return RAS_EINVAL; }
    if (opts.pou != RAS_POU_LINEAR && opts.pou != RAS_POU_BOOLEAN) { err = "unknown pou"; return RAS_EINVAL; }
    if (opts.precision != RAS_MIXED && opts.precision != RAS_FP64) { err = "unknown precision"; return RAS_EINVAL; }
    if (bad(opts.sigma)) { err = "sigma must be finite"; return RAS_EINVAL; }
    const int G = opts.global_pml < 0 ? pml_width : opts.global_pml;
    const int n_int = grid[0];
    const long long Ncl = static_cast<long long>(n_int) + 2LL * G;
    if (Ncl < 2 || Ncl > 200000) { err = "mesh size out of range"; return RAS_EINVAL; }
    const int Nc = static_cast<int>(Ncl);
    const int Px = subdomains[0], Py = subdomains[1];
    if (Px < 1 || Py < 1 || Px > Nc || Py > Nc) {
        err = "subdomains per side must be between 1 and the number of cells";
        return RAS_EINVAL;
    }

    out.k = k;
    out.h = h;
    out.sigma = opts.sigma > 0.0 ? opts.sigma : 10.0 * k;
    out.n_int = n_int;
    out.G = G;
    out.Nc = Nc;
    out.Px = Px;
    out.Py = Py;
    out.delta = overlap;
    out.kappa = pml_width;
    out.bc = opts.bc;
    out.pou = opts.pou;
    out.ndof = static_cast<long long>(Nc - 1) * (Nc - 1);

    std::vector<Axis> ax(Px), ay(Py);
    for (int p = 0; p < Px; ++p) ax[p] = make_axis(Nc, Px, p, overlap, pml_width, opts.bc);
    for (int q = 0; q < Py; ++q) ay[q] = make_axis(Nc, Py, q, overlap, pml_width, opts.bc);
    if (!pou_axis(ax, Nc, overlap, opts.pou, out.pou_cnt[0], out.pou_chunk[0], out.pou_w[0]) ||
        !pou_axis(ay, Nc, overlap, opts.pou, out.pou_cnt[1], out.pou_chunk[1], out.pou_w[1])) {
        err = "more than 4 overlapping subdomains at one node; use fewer subdomains or a smaller overlap";
        return RAS_ENOTSUP;
    }
    // every node where chi_j > 0 must be an unknown of subdomain j
    for (int axis = 0; axis < 2; ++axis) {
        const std::vector<Axis> &A = axis == 0 ? ax : ay;
        for (int i = 1; i < Nc; ++i) {
            for (int e = 0; e < out.pou_cnt[axis][i]; ++e) {
                const Axis &a = A[out.pou_chunk[axis][static_cast<size_t>(i) * kMaxPou + e]];
                if (i < a.u_lo || i > a.u_hi) {
                    err = "the partition of unity is non-zero at a node that is not a local "
                          "unknown (Dirichlet subdomains need an overlap or a PML)";
                    return RAS_EINVAL;
                }
            }
        }
    }

    out.subs.clear();
    out.subs.reserve(static_cast<size_t>(Px) * Py);
    for (int q = 0; q < Py; ++q) {
        for (int p = 0; p < Px; ++p) {
            const Axis &a = ax[p], &b = ay[q];
            DevSub s{};
            s.nx = a.u_hi - a.u_lo + 1;
            s.ny = b.u_hi - b.u_lo + 1;
            if (s.nx < 1 || s.ny < 1) {
                err = "a subdomain has no unknowns";
                return RAS_EINVAL;
            }
            s.ix0 = a.u_lo;
            s.jy0 = b.u_lo;
            s.xfast = s.nx <= s.ny ? 1 : 0;
            s.nf = s.xfast ? s.nx : s.ny;
            s.W = (s.nf + 3) & ~1;    // nf + 2, rounded up to even (one zero slot)
            if (s.W > kMaxW) s.W = (s.nf + 2 + 63) / 64 * 64;    // the wide kernels' ring
            if (s.W > kMaxWideW) {
                std::snprintf(buf, sizeof buf,
                              "subdomain band %d exceeds the supported maximum %d; use more subdomains",
                              s.nf + 1, kMaxWideW - 1);
                err = buf;
                return RAS_ENOTSUP;
            }
            s.n = s.nx * s.ny;
            s.npad = (s.n + kPad - 1) / kPad * kPad;
            s.bx0 = a.box_lo;
            s.bx1 = a.box_hi;
            s.by0 = b.box_lo;
            s.by1 = b.box_hi;
            s.flags = (a.pml_lo ? SD_PML_XLO : 0) | (a.pml_hi ? SD_PML_XHI : 0) |
                      (b.pml_lo ? SD_PML_YLO : 0) | (b.pml_hi ? SD_PML_YHI : 0) |
                      (a.imp_lo ? SD_IMP_XLO : 0) | (a.imp_hi ? SD_IMP_XHI : 0) |
                      (b.imp_lo ? SD_IMP_YLO : 0) | (b.imp_hi ? SD_IMP_YHI : 0);
            s.ax = (a.int_lo - G) * h;
            s.bx = (a.int_hi - G) * h;
            s.ay = (b.int_lo - G) * h;
            s.by = (b.int_hi - G) * h;
            s.prob = 0;
            s.cp = p;
            s.cq = q;
            s.ix_int0 = a.int_lo;
            s.ix_int1 = a.int_hi;
            s.iy_int0 = b.int_lo;
            s.iy_int1 = b.int_hi;
            out.subs.push_back(s);
        }
    }
    return RAS_OK;
}

void desc_ints(const DevSub &s, const PlanProblem &pb, int *o) {
    for (int i = 0; i < RAS_DESC_INTS; ++i) o[i] = 0;
    o[0] = s.n;
    o[1] = s.nf;
    o[2] = s.W;
    o[3] = s.xfast;
    o[4] = s.ix0;
    o[5] = s.nx;
    o[6] = s.jy0;
    o[7] = s.ny;
    o[8] = s.cp;
    o[9] = s.cq;
    o[10] = s.ix_int0;
    o[11] = s.ix_int1;
    o[12] = s.iy_int0;
    o[13] = s.iy_int1;
    o[14] = s.bx0;
    o[15] = s.bx1;
    o[16] = s.by0;
    o[17] = s.by1;
    o[18] = s.flags;
    o[19] = s.prob;
    o[20] = pb.delta;
    o[21] = pb.kappa;
    o[22] = pb.G;
}

// Section 3 (iii): a layer of C l(k) wavelengths, with the slowly growing
// factor l(k) = k/(k - k0) log2(k/k0), which tends to 1/ln 2 as k -> k0 (the
// removable singularity is evaluated through log1p of (k - k0)/k0 near it),
// converted to whole mesh cells by rounding down.  A relative slack of 1e-9
// keeps a width that is an exact multiple of h from dropping a cell.
int width_rule_cells(double k, double h, double C, double k0, int &cells, std::string &err) {
    if (bad(k) || k <= 0.0 || bad(h) || h <= 0.0 || bad(k0) || k0 <= 0.0 || bad(C) || C < 0.0) {
        err = "width rule needs finite k, h, k0 > 0 and C >= 0";
        return RAS_EINVAL;
    }
    const double t = (k - k0) / k0;              // k/k0 = 1 + t
    double ell;
    if (std::fabs(t) < 1e-6)                     // series of log1p(t)/t about t = 0
        ell = (1.0 + t) * (1.0 - t / 2.0 + t * t / 3.0) / std::log(2.0);
    else
        ell = (1.0 + t) / t * std::log1p(t) / std::log(2.0);
    const double cells_real = C * ell * (2.0 * M_PI / k) / h;
    if (!(cells_real < 1e9)) { err = "width rule: width exceeds 1e9 cells"; return RAS_EINVAL; }
    cells = static_cast<int>(std::floor(cells_real * (1.0 + 1e-9)));
    return RAS_OK;
}

}  // namespace raspml
