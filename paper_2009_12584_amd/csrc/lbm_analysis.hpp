// Drop-shape diagnostics shared by the single and batched entry points.
#pragma once

#include "lbm_common.hpp"

namespace mclbm {

// Contour circle fit (lbm_analysis.hip): workgroups of the moment pass, the
// largest wall-distance cut, and the device work buffer it needs in doubles.
constexpr int CONTOUR_BLOCKS = 1024;
constexpr int CONTOUR_MAX_SKIP = 32;
constexpr size_t CONTOUR_WORK_DOUBLES = (size_t)CONTOUR_BLOCKS * 10 + 8;

// Circle through the interface rho^A = q->level of the FP32 density field
// rhoA (nx * ny, unpadded) with classification cls; enqueued on s, then
// synchronises and fills *out.  work: CONTOUR_WORK_DOUBLES device doubles.
int contour_fit(const float *rhoA, const uint8_t *cls, int nx, int ny, const lbm_contour_req *q, double *work,
                hipStream_t s, lbm_circle_t *out);

// Interface crossing along a lattice line into the device double *out
// (enqueued on s, no synchronisation); line_probe_check is its host-side
// argument check, also usable before any device work is enqueued.
int line_probe_check(int nx, int ny, int x0, int y0, int dx, int dy, int len, double level, const double *out);
int line_probe(const float *rhoA, const uint8_t *cls, int nx, int ny, int x0, int y0, int dx, int dy, int len,
               double level, double *out, hipStream_t s);

}  // namespace mclbm
