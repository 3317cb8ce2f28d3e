// FP64 vector kernels of the Davidson solver.  Reductions are two-pass
// (per-block partial sums, then a fixed-order sum), so results are bitwise
// reproducible.
#include <hip/hip_runtime.h>
#include "davidson.hpp"

namespace dmrg {

constexpr int VB = 256;          // threads per block
constexpr int VCHUNK = 4096;     // vector elements per block in the dot kernel

// part[b * m + j] = sum_{i in chunk b} V[j * ldv + i] * x[i], j < m
__global__ void __launch_bounds__(VB) dots_kernel(const double *__restrict__ V, int64_t ldv, int m,
                                                   const double *__restrict__ x, int64_t n,
                                                   double *__restrict__ part) {
  __shared__ double red[VB];
  const int64_t i0 = (int64_t)blockIdx.x * VCHUNK;
  const int64_t i1 = min(n, i0 + VCHUNK);
  for (int j = 0; j < m; j++) {
    double acc = 0.0;
    const double *v = V + (int64_t)j * ldv;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += VB) acc += v[i] * x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = VB / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * m + j] = red[0];
    __syncthreads();
  }
}

// out[j] = sum_b part[b * m + j], in block order
__global__ void dots_finish_kernel(const double *__restrict__ part, int nb, int m, double *__restrict__ out) {
  int j = threadIdx.x;
  if (j < m) {
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += part[(int64_t)b * m + j];
    out[j] = s;
  }
}

// y[i] = beta * y[i] + sign * sum_j c[j] V[j * ldv + i]   (c on the device)
__global__ void __launch_bounds__(VB) combo_kernel(const double *__restrict__ V, int64_t ldv, int m,
                                                    const double *__restrict__ c, double sign, double beta,
                                                    double *__restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
    double acc = 0.0;
    for (int j = 0; j < m; j++) acc += c[j] * V[(int64_t)j * ldv + i];
    y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + sign * acc;
  }
}

// r = hu - theta u ; t = -r / (diag - theta) with |denominator| >= floor
__global__ void __launch_bounds__(VB) resid_kernel(const double *__restrict__ hu, const double *__restrict__ u,
                                                    const double *__restrict__ diag, double theta, double floor_,
                                                    double *__restrict__ r, double *__restrict__ t, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) {
    double ri = hu[i] - theta * u[i];
    double d = diag[i] - theta;
    if (fabs(d) < floor_) d = d < 0.0 ? -floor_ : floor_;
    r[i] = ri;
    t[i] = -ri / d;
  }
}

// x *= s
__global__ void __launch_bounds__(VB) scale_kernel(double *__restrict__ x, double s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB) x[i] *= s;
}

static int vgrid(int64_t n) { return (int)std::min<int64_t>((n + VB - 1) / VB, 8192); }

void vec_dots(const double *V, int64_t ldv, int m, const double *x, int64_t n, double *part, double *out,
              void *stream) {
  int nb = (int)((n + VCHUNK - 1) / VCHUNK);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(VB), 0, (hipStream_t)stream, V, ldv, m, x, n, part);
  hipLaunchKernelGGL(dots_finish_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, part, nb, m, out);
}

int64_t vec_dots_part_len(int64_t n, int m) { return ((n + VCHUNK - 1) / VCHUNK + 1) * (int64_t)m; }

void vec_combo(const double *V, int64_t ldv, int m, const double *c, double sign, double beta, double *y,
               int64_t n, void *stream) {
  hipLaunchKernelGGL(combo_kernel, dim3(vgrid(n)), dim3(VB), 0, (hipStream_t)stream, V, ldv, m, c, sign, beta, y,
                     n);
}

void vec_resid(const double *hu, const double *u, const double *diag, double theta, double floor_, double *r,
               double *t, int64_t n, void *stream) {
  hipLaunchKernelGGL(resid_kernel, dim3(vgrid(n)), dim3(VB), 0, (hipStream_t)stream, hu, u, diag, theta, floor_,
                     r, t, n);
}

void vec_scale(double *x, double s, int64_t n, void *stream) {
  hipLaunchKernelGGL(scale_kernel, dim3(vgrid(n)), dim3(VB), 0, (hipStream_t)stream, x, s, n);
}

}  // namespace dmrg
