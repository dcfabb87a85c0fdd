// mpm_tune.h -- launch shapes picked at run time (mpm_autotune).
#pragma once

#include <stdint.h>

namespace mpm {

// Workgroup target of CG sweep A for a grid of nx x ny x nz: the one
// mpm_autotune picked for exactly that size in this process, else the
// built-in choice.
int tall_target(int64_t nx, int64_t ny, int64_t nz);

// Workgroup target of the column walks (JTV weights, halved-step acceptance)
// for that grid: the one set by mpm_autotune_set, else the built-in choice.
int column_target(int64_t nx, int64_t ny, int64_t nz);

}  // namespace mpm
