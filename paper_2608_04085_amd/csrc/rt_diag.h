// Internal launch interface of the diagnostic reductions (rt_diag.hip).
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

// Widest row (and, for the 2-D spectrum, tallest column) the spectrum
// kernels take: their twiddle tables (2 nx doubles) live in LDS.
constexpr int kSpecMaxNx = 4096;

// E[b][n] = sum over the selected rows of |sum_x f_b(j, x) e^{-2 pi i n x / nx}|^2
// for n = 0 .. nx/2; member b's field starts at f + b * member_stride, rows of
// nx doubles; row = -1 selects every row.
hipError_t launch_row_spectrum(int nx, int ny, int nb, const double* f, long long member_stride, int row, double* E,
                               hipStream_t s);

// E[b][q][k] = |F_b(q, k)|^2, F_b(q, k) = sum_{y, x} f_b(y, x)
// e^{-2 pi i (k x / nx + q y / ny)}, for q = 0 .. ny - 1, k = 0 .. nx/2 (the
// half plane of a real field); C holds 2 nb ny (nx/2 + 1) doubles of
// scratch (the row transforms).
hipError_t launch_power_spectrum_2d(int nx, int ny, int nb, const double* f, long long member_stride, double* C,
                                    double* E, hipStream_t s);

}  // namespace rtk
