// Diagnostics of a march that read a field once and reduce it: the
// horizontal power spectrum of Eq. 12 and the 2-D power spectrum whose
// strongest modes make the 90 %-power reconstruction of App. B.  Kept apart from the stepping
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

// 2-D DFT, pass 1: C[b][y][k] = sum_x f_b(y, x) e^{-2 pi i k x / nx} for
// k = 0 .. nx/2, as (re, im) pairs.  One thread per coefficient, threads of
// a block along k for one row (the row's values are read by every thread:
// broadcast), twiddles in LDS.
__global__ __launch_bounds__(kSpecThreads) void k_dft_rows(int nx, int ny, const double* f, long long mstride,
                                                           int nk, double* C) {
  extern __shared__ double tw[];  // [0, nx): cos(2 pi k / nx), [nx, 2 nx): sin
  const int y = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  for (int k = tid; k < nx; k += kSpecThreads) {
    double sn, cs;
    sincospi(2.0 * k / nx, &sn, &cs);
    tw[k] = cs;
    tw[nx + k] = sn;
  }
  __syncthreads();
  const int k = blockIdx.x * kSpecThreads + tid;
  if (k >= nk) return;
  const double* fr = f + (long long)b * mstride + (size_t)y * nx;
  double re = 0.0, im = 0.0;
  int idx = 0;
  for (int x = 0; x < nx; ++x) {
    const double v = fr[x];
    re += v * tw[idx];
    im -= v * tw[nx + idx];
    idx += k;
    if (idx >= nx) idx -= nx;
  }
  double* c = C + (((size_t)b * ny + y) * nk + k) * 2;
  c[0] = re;
  c[1] = im;
}

// Pass 2: F[b][q][k] = sum_y C[b][y][k] e^{-2 pi i q y / ny} for q = 0 ..
// ny - 1, and E = |F|^2.  One thread per (q, k), threads of a block along q
// for one k (each C[y][k] is read by every thread: broadcast).
__global__ __launch_bounds__(kSpecThreads) void k_dft_cols_power(int ny, int nk, const double* C, double* E) {
  extern __shared__ double tw[];  // [0, ny): cos(2 pi q / ny), [ny, 2 ny): sin
  const int k = blockIdx.y, b = blockIdx.z, tid = threadIdx.x;
  for (int q = tid; q < ny; q += kSpecThreads) {
    double sn, cs;
    sincospi(2.0 * q / ny, &sn, &cs);
    tw[q] = cs;
    tw[ny + q] = sn;
  }
  __syncthreads();
  const int q = blockIdx.x * kSpecThreads + tid;
  if (q >= ny) return;
  const double* cb = C + (size_t)b * ny * nk * 2 + (size_t)k * 2;
  double re = 0.0, im = 0.0;
  int idx = 0;
  for (int y = 0; y < ny; ++y) {
    const double cr = cb[(size_t)y * nk * 2], ci = cb[(size_t)y * nk * 2 + 1];
    const double c = tw[idx], s = tw[ny + idx];
    // (cr + i ci)(c - i s)
    re += cr * c + ci * s;
    im += ci * c - cr * s;
    idx += q;
    if (idx >= ny) idx -= ny;
  }
  E[((size_t)b * ny + q) * nk + k] = re * re + im * im;
}

}  // namespace

hipError_t launch_power_spectrum_2d(int nx, int ny, int nb, const double* f, long long member_stride, double* C,
                                    double* E, hipStream_t s) {
  if (nx < 1 || nx > kSpecMaxNx || ny < 1 || ny > kSpecMaxNx || nb < 1) return hipErrorInvalidValue;
  const int nk = nx / 2 + 1;
  hipLaunchKernelGGL(k_dft_rows, dim3((nk + kSpecThreads - 1) / kSpecThreads, ny, nb), dim3(kSpecThreads),
                     2 * (size_t)nx * sizeof(double), s, nx, ny, f, member_stride, nk, C);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dft_cols_power, dim3((ny + kSpecThreads - 1) / kSpecThreads, nk, nb), dim3(kSpecThreads),
                     2 * (size_t)ny * sizeof(double), s, ny, nk, C, E);
  return hipGetLastError();
}

hipError_t launch_row_spectrum(int nx, int ny, int nb, const double* f, long long member_stride, int row, double* E,
                               hipStream_t s) {
  if (nx < 1 || nx > kSpecMaxNx || ny < 1 || nb < 1 || row < -1 || row >= ny) return hipErrorInvalidValue;
  const int nbins = nx / 2 + 1;
  hipLaunchKernelGGL(k_row_spectrum, dim3(nbins, nb), dim3(kSpecThreads), 2 * (size_t)nx * sizeof(double), s, nx,
                     ny, f, member_stride, row, nbins, E);
  return hipGetLastError();
}

}  // namespace rtk
