// Diagnostics of a march that read a field once and reduce it: the
// horizontal power spectrum of Eq. 12.  Kept apart from the stepping
// kernels; launched through rt_diag.h by the C ABI.
#include <hip/hip_runtime.h>

#include "rt_diag.h"

namespace rtk {
namespace {

constexpr int kSpecThreads = 256;

// One block per (mode n, member b): each thread takes whole rows of the
// selection, forms the row's Fourier coefficient at n with the twiddles
// exp(-2 pi i k / nx) held in LDS (index n x mod nx, advanced by n per
// column), and accumulates its squared modulus; a fixed-order tree sums
// the threads.
__global__ __launch_bounds__(kSpecThreads) void k_row_spectrum(int nx, int ny, const double* f, long long mstride,
                                                               int row, int nbins, double* E) {
  extern __shared__ double tw[];  // [0, nx): cos(2 pi k / nx), [nx, 2 nx): sin
  __shared__ double red[kSpecThreads];
  const int n = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  for (int k = tid; k < nx; k += kSpecThreads) {
    double s, c;
    sincospi(2.0 * k / nx, &s, &c);
    tw[k] = c;
    tw[nx + k] = s;
  }
  __syncthreads();
  const double* fb = f + (long long)b * mstride;
  const int j0 = row < 0 ? 0 : row, j1 = row < 0 ? ny : row + 1;
  double acc = 0.0;
  for (int j = j0 + tid; j < j1; j += kSpecThreads) {
    const double* fr = fb + (size_t)j * nx;
    double re = 0.0, im = 0.0;
    int idx = 0;
    for (int x = 0; x < nx; ++x) {
      const double v = fr[x];
      re += v * tw[idx];
      im -= v * tw[nx + idx];
      idx += n;
      if (idx >= nx) idx -= nx;
    }
    acc += re * re + im * im;
  }
  red[tid] = acc;
  __syncthreads();
  for (int s = kSpecThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) E[(size_t)b * nbins + n] = red[0];
}

}  // namespace

hipError_t launch_row_spectrum(int nx, int ny, int nb, const double* f, long long member_stride, int row, double* E,
                               hipStream_t s) {
  if (nx < 1 || nx > kSpecMaxNx || ny < 1 || nb < 1 || row < -1 || row >= ny) return hipErrorInvalidValue;
  const int nbins = nx / 2 + 1;
  hipLaunchKernelGGL(k_row_spectrum, dim3(nbins, nb), dim3(kSpecThreads), 2 * (size_t)nx * sizeof(double), s, nx,
                     ny, f, member_stride, row, nbins, E);
  return hipGetLastError();
}

}  // namespace rtk
