// Broadband dirty map with the band's bins summed first (Sec. V): per segment a
// table of Y_t(tau) = sum_k y(t,k) e^{2 pi i (f_k - f_c) tau} on the delay grid
// tau_j = (j - m - 1) h, j < G = 2m + 3, read by 4-point Lagrange interpolation;
// and the broadband entry that picks between it and the strip sums of the
// matrix-core dirty map.
#pragma once

#include "sgwb_internal.h"

namespace sgwb {

struct BbGrid {
    int32_t m = 0, G = 0;
    double h = 0.0;      // node spacing (s)
    double bound = 0.0;  // the seeds' promised bound on |tau| (s), <= m h
};
// false: no grid of at most 2^21 + 3 nodes meets the spacing for this band
bool bb_grid(int32_t nb, double df, double bound, BbGrid *g);
size_t bb_workspace_bytes(int32_t nt, int32_t npix, int32_t nb, const BbGrid &g);

// The layout of launch_band_gamma's work (band.hip), for a pass that computes
// Gbb beside Xbb with the same bits: its scratch holds v[nt] (the band-summed
// weights, from launch_band_weights) and then band_gamma_chunks() rows of
// per-pixel partial sums, row r over segments [r per, (r + 1) per),
// per = ceil(nt / band_gamma_chunks()), each summed in segment order.
int32_t band_gamma_chunks();
hipError_t launch_band_weights(const float *w, int64_t ldw, int32_t nt, const float *H, int32_t klo, int32_t khi,
                               double *v, hipStream_t s);
// Xbb (and, with Gbb, Gbb) over columns [klo, khi) of C and w (absolute bins
// k0 + klo ..); H is needed with Gbb
// nside > 0: antipodal seeds (spot-checked), one thread per pixel pair
hipError_t launch_broadband_table_maps(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t klo,
                                       int32_t khi, double f0, double df, int64_t k0, const float *H,
                                       const float *gamma, const double *tau, int32_t npix, int64_t nside,
                                       const BbGrid &g, float *Xbb, float *Gbb, void *work, hipStream_t s);

// The host's cost estimate (s) of the route sgwb_broadband_maps takes for
// these arguments; -1 where it would refuse them.
double broadband_cost_seconds(int32_t nt, int32_t nf, int32_t npix, uint32_t flags, const sgwb_fgrid *fg,
                              int32_t k_lo, int32_t k_hi, double tau_bound);

// sgwb_broadband_maps with the strips route's seed-side products from `seeds`
// (as make_maps_band_seeded; the table route needs none).
int broadband_maps_seeded(const float *C, const float *w, int64_t ldc, int32_t nt, int32_t nf, const sgwb_fgrid *fg,
                          int64_t k0, const float *gamma, const double *tau, int32_t npix, uint32_t flags,
                          double tau_bound, const float *H, int32_t k_lo, int32_t k_hi, float *Xbb, float *Gbb,
                          void *workspace, size_t workspace_bytes, const void *seeds, hipStream_t stream);

}  // namespace sgwb
