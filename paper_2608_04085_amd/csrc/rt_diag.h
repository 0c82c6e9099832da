// Internal launch interface of the diagnostic reductions (rt_diag.hip).
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

// Widest row the spectrum kernel takes: its twiddle table (2 nx doubles)
// lives in LDS.
constexpr int kSpecMaxNx = 4096;

// E[b][n] = sum over the selected rows of |sum_x f_b(j, x) e^{-2 pi i n x / nx}|^2
// for n = 0 .. nx/2; member b's field starts at f + b * member_stride, rows of
// nx doubles; row = -1 selects every row.
hipError_t launch_row_spectrum(int nx, int ny, int nb, const double* f, long long member_stride, int row, double* E,
                               hipStream_t s);

}  // namespace rtk
