// adaptive.h -- the adaptive line windows' per-cell buffer and the
// wing-return launch (internal; see adaptive.hip).
#pragma once

#include "rt_internal.h"

namespace rt {

// Doubles per cell in ctx->d_sbar: sbar and the partition ratio (2), the
// screening's 8-float cell record (4), then the wing-return constant (1).
constexpr int kAdaptiveCellDoubles = 7;

// The wing-return constants, one per cell, FP64, in cm^-1: the last of the
// per-cell segments.
inline double* adaptive_wing_constants(rt_ctx c) {
  return c->d_sbar + (kAdaptiveCellDoubles - 1) * c->n_cells;
}

// RT_KAPPA_ADAPTIVE_WINGS: the adaptive windows, then per cell the
// midpoint-rule mass of the dropped points spread over the band, added to
// every point of the line sum.
hipError_t launch_kappa_adaptive_wings(rt_ctx c);

}  // namespace rt
