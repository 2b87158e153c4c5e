// Full Fisher matrix for general weights (Eq. eq_fisher with any w(t,c), the
// broadband H weighting of Sec. V): one delay table per segment, built on the
// float64 matrix cores, then the matrix from those tables (fisher_full.hip).
#pragma once

#include "sgwb_internal.h"

namespace sgwb {

// w[nt][ldw], column c = bin k0 + c; the workspace layout depends on nside
// (0: every pixel a row and a column; > 0: the antipodal blocks).
size_t fisher_full_general_workspace_bytes(double f0, double df, int64_t k0, int32_t clo, int32_t chi, int32_t nt,
                                           int32_t npix, int64_t nside);
hipError_t launch_fisher_full_general(const float *w, int64_t ldw, const float *H, int32_t clo, int32_t chi,
                                      double f0, double df, int64_t k0, const float *gamma, const double *tau,
                                      int32_t nt, int32_t npix, int64_t nside, float *G, void *work, hipStream_t s);

}  // namespace sgwb
