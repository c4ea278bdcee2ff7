// Column-scaled sums of device blocks (the inverse iterations' right-hand sides).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bemrat {

// out[r][c] = sum_{b < nb} coef[b][c] X_b[r][c] (fixed order b = 0, 1, ...), r < n, c < m,
// nb <= kBlockCombineMax; blocks [host] holds nb device pointers to n x m blocks of row
// stride ldx, coef is device nb x m, out device n x m of row stride ldo.
constexpr int kBlockCombineMax = 64;
hipError_t launch_block_combine(const double2 *const *blocks, int nb, const double2 *coef, int64_t n, int64_t m,
                                int64_t ldx, double2 *out, int64_t ldo, hipStream_t stream);

}  // namespace bemrat
