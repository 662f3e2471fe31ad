// Learned warm start: internal interface between the network object
// (warm_net.hip), its kernels (k_warm.hip) and the solver handle (abi.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "ras_pml.h"

namespace raspml {

// learned warm start (warm_net.hip, k_warm.hip)
int wsnet_forward(ras_pml_wsnet *N, const float *x, int B, float *out, hipStream_t st);
int wsnet_grid(const ras_pml_wsnet *N);
float *wsnet_stage(ras_pml_wsnet *N);
float *wsnet_out(ras_pml_wsnet *N);
void warm_grid_sample(const double2 *vec, int n1, int G, int grid, double scale, float *out,
                      hipStream_t s);
void warm_grid_scatter(const float *in, int n1, int G, int grid, double scale, double2 *vec,
                       long long ndof, hipStream_t s);

}  // namespace raspml
