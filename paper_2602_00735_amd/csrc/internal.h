// Internal data structures shared by the host planner, the kernels and the
// C ABI.  Plain structs: the device reads them as they are laid out here.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ras_pml.h"

namespace raspml {

// Factor column length W: n_fast + 2 rounded up to even up to kMaxW (the
// register-ring kernels), else rounded up to a multiple of 64 up to
// kMaxWideW (the wide kernels: 3 to 7 registers of 64 slots per lane).
constexpr int kMaxW = 128;
constexpr int kMaxWideW = 448;
// Largest number of chunks whose partition-of-unity weight is non-zero at
// one mesh node along one axis.
constexpr int kMaxPou = 4;
// Local vectors and factor columns are padded to a multiple of this.
constexpr int kPad = 64;
// The band solve reads each subdomain's factor as one stream and prefetches
// up to 32 vectors (at most 32 KB) past its end; the factor allocation ends
// with this much slack so that the last subdomain's over-read stays inside.
constexpr int kFactorSlack = 65536;

// Flags of a subdomain descriptor.
enum : int {
    SD_PML_XLO = 1, SD_PML_XHI = 2, SD_PML_YLO = 4, SD_PML_YHI = 8,
    SD_IMP_XLO = 16, SD_IMP_XHI = 32, SD_IMP_YLO = 64, SD_IMP_YHI = 128
};

// One subdomain, as the kernels see it.
struct DevSub {
    int n;          // local unknowns
    int npad;       // n rounded up to kPad
    int nf;         // unknowns along the fast axis
    int W;          // factor column length: half-bandwidth + 1 = nf + 2, rounded
                    // up to even (the extra slot holds zeros); above kMaxW
                    // rounded up to a multiple of 64 (the wide kernels)
    int xfast;      // 1: x is the fast axis
    int ix0, nx;    // first unknown node index and count along x
    int jy0, ny;    // same along y
    int prob;       // problem index
    int bx0, bx1, by0, by1;   // Omega_j box in node indices
    int flags;      // SD_* bits
    int cp, cq;     // chunk indices along x and y
    int ix_int0, ix_int1, iy_int0, iy_int1;   // Omega_{j,int} in node indices
    int pad_;
    double ax, bx, ay, by;    // Omega_{j,int} edges (coordinates)
    long long fac_off;  // first L entry (elements); D^{-1} follows npad*W later
    long long vec_off;  // first entry of this subdomain's padded local vectors
    long long loc_off;  // first entry in the unpadded back-to-back layout
    // the PoU sum's view, one 16-byte load: node (i, j) of the problem is
    // entry pou_off + i pou_sx + j pou_sy of the padded local vectors
    int pou_off, pou_sx, pou_sy, pou_pad_;
};
static_assert(sizeof(DevSub) % 16 == 0 && offsetof(DevSub, pou_off) % 16 == 0,
              "DevSub: the PoU sum reads pou_off .. pou_pad_ as one 16-byte load");

// One problem, as the kernels see it.
struct DevProb {
    double k, h, sigma;
    int G, Nc, n1;        // n1 = Nc - 1 unknowns per side
    int Px, Py;
    int sub_first;        // first subdomain index of this problem
    int pou_x, pou_y;     // offsets into the PoU tables (in nodes)
    int pad_;
    long long dof_off;    // first unknown in the concatenated vectors
    long long ndof;
};

// Per-problem GMRES state kept on the device.
struct KState {
    double bnorm;      // ||b||
    double beta;       // ||r0|| of the current cycle
    double est;        // |g_{j+1}| after the last step
    double rtol;
    int kp;            // Arnoldi steps taken in the current cycle (the index
                       // of the next step's Krylov vector)
    int in_cycle;      // 1 while the problem takes steps in this cycle
    int breakdown;     // Arnoldi broke down in this cycle
    int mc;            // steps this cycle may take (<= restart)
};

// Per-problem state of the fixed-point iteration kept on the device.
struct RState {
    double bnorm;      // ||b||
    double relres;     // ||b - A x|| / ||b|| of the current iterate
    int iters;         // steps taken
    int nonfinite;     // the residual stopped being finite
};

// One block of the fused Arnoldi-step kernel: a contiguous slice of one
// problem's unknowns.
struct ArnoldiBlock {
    int prob;        // problem of this block
    int first_blk;   // first block of that problem
    int nblk;        // blocks of that problem
    int n;           // unknowns of this block (<= 256 E)
    long long first; // first unknown (index into the concatenated vectors)
};

// Host-side plan of one problem.
struct PlanProblem {
    double k, h, sigma;
    int n_int, G, Nc, Px, Py, delta, kappa, bc, pou;
    long long ndof;
    std::vector<DevSub> subs;          // q * Px + p order
    // 1D partition of unity along each axis: for node i (0..Nc) up to
    // kMaxPou (chunk, weight) pairs with weight > 0.
    std::vector<int> pou_cnt[2];
    std::vector<int> pou_chunk[2];     // (Nc+1) * kMaxPou
    std::vector<double> pou_w[2];      // (Nc+1) * kMaxPou
};

// Validate one problem and compute its subdomains and PoU tables.
// Returns RAS_OK or an error status with a message in `err`.
int width_rule_cells(double k, double h, double C, double k0, int &cells, std::string &err);
int plan_problem(double k, double h, const int grid[2], const int subdomains[2],
                 int overlap, int pml_width, const ras_pml_opts &opts,
                 PlanProblem &out, std::string &err);

// Descriptor in the int32 layout documented in ras_pml.h.
void desc_ints(const DevSub &s, const PlanProblem &pb, int *out);

}  // namespace raspml
