// FP64 vector kernels of the Davidson solver.  Vectors are concatenations of
// one segment per problem; work is cut into chunks that never cross a
// segment, and every reduction is two-pass (per-chunk partial sums, then a
// fixed-order sum per segment), so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include "davidson.hpp"

namespace dmrg {

constexpr int VB = 256;          // threads per block

// part[c * m + j] = sum_{i in chunk c} V[j * ldv + i] * x[i], j < m
__global__ void __launch_bounds__(VB) sdots_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                    const double *__restrict__ V, int64_t ldv, int m,
                                                    const double *__restrict__ x, double *__restrict__ part) {
  __shared__ double red[VB];
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    for (int j = 0; j < m; j++) {
      double acc = 0.0;
      const double *v = V + (int64_t)j * ldv;
      for (int64_t i = C.i0 + threadIdx.x; i < C.i1; i += VB) acc += v[i] * x[i];
      red[threadIdx.x] = acc;
      __syncthreads();
      for (int s = VB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[(int64_t)c * m + j] = red[0];
      __syncthreads();
    }
  }
}

// out[k * m + j] = sum of the partials of segment k's chunks, in chunk order
__global__ void sdots_finish_kernel(const int32_t *__restrict__ seg_chunk0, int nseg, int m,
                                    const double *__restrict__ part, double *__restrict__ out) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nseg * m; t += gridDim.x * blockDim.x) {
    int k = t / m, j = t - k * m;
    double s = 0.0;
    for (int c = seg_chunk0[k]; c < seg_chunk0[k + 1]; c++) s += part[(int64_t)c * m + j];
    out[t] = s;
  }
}

// y[i] = beta y[i] + sign * sum_j coef[k * ldc + j] V[j * ldv + i]   (k = segment of i)
__global__ void __launch_bounds__(VB) scombo_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                     const double *__restrict__ V, int64_t ldv, int m,
                                                     const double *__restrict__ coef, int ldc, double sign,
                                                     double beta, double *__restrict__ y) {
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    const double *cf = coef + (int64_t)C.seg * ldc;
    for (int64_t i = C.i0 + threadIdx.x; i < C.i1; i += VB) {
      double acc = 0.0;
      for (int j = 0; j < m; j++) acc += cf[j] * V[(int64_t)j * ldv + i];
      y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + sign * acc;
    }
  }
}

// r = hu - theta_k u ; t = -r / (diag - theta_k) with |denominator| >= floor
__global__ void __launch_bounds__(VB) sresid_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                     const double *__restrict__ hu, const double *__restrict__ u,
                                                     const double *__restrict__ diag,
                                                     const double *__restrict__ theta, double floor_,
                                                     double *__restrict__ r, double *__restrict__ t) {
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    const double th = theta[C.seg];
    for (int64_t i = C.i0 + threadIdx.x; i < C.i1; i += VB) {
      double ri = hu[i] - th * u[i];
      double d = diag[i] - th;
      if (fabs(d) < floor_) d = d < 0.0 ? -floor_ : floor_;
      r[i] = ri;
      t[i] = -ri / d;
    }
  }
}

// x[i] *= s_k
__global__ void __launch_bounds__(VB) sscale_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                     const double *__restrict__ s, double *__restrict__ x) {
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    const double f = s[C.seg];
    for (int64_t i = C.i0 + threadIdx.x; i < C.i1; i += VB) x[i] *= f;
  }
}

// x[i] = value
__global__ void __launch_bounds__(VB) sfill_kernel(const VChunk *__restrict__ chunks, int nchunks, double value,
                                                    double *__restrict__ x) {
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    for (int64_t i = C.i0 + threadIdx.x; i < C.i1; i += VB) x[i] = value;
  }
}

// dst[i] = src[i] where the segment's flag is non-zero
__global__ void __launch_bounds__(VB) sselect_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                      const double *__restrict__ flag, const double *__restrict__ src,
                                                      double *__restrict__ dst) {
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    if (flag[C.seg] == 0.0) continue;
    for (int64_t i = C.i0 + threadIdx.x; i < C.i1; i += VB) dst[i] = src[i];
  }
}

static int cgrid(int nchunks) { return std::min(std::max(nchunks, 1), 16384); }

void vec_dots(const VecCtx &X, const double *V, int64_t ldv, int m, const double *x, double *out, void *stream) {
  hipLaunchKernelGGL(sdots_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     V, ldv, m, x, X.part);
  int tot = X.nseg * m;
  hipLaunchKernelGGL(sdots_finish_kernel, dim3(std::max(1, (tot + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     X.seg_chunk0, X.nseg, m, X.part, out);
}

void vec_combo(const VecCtx &X, const double *V, int64_t ldv, int m, const double *coef, int ldc, double sign,
               double beta, double *y, void *stream) {
  hipLaunchKernelGGL(scombo_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     V, ldv, m, coef, ldc, sign, beta, y);
}

void vec_resid(const VecCtx &X, const double *hu, const double *u, const double *diag, const double *theta,
               double floor_, double *r, double *t, void *stream) {
  hipLaunchKernelGGL(sresid_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     hu, u, diag, theta, floor_, r, t);
}

void vec_scale(const VecCtx &X, const double *s, double *x, void *stream) {
  hipLaunchKernelGGL(sscale_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     s, x);
}

void vec_fill(const VecCtx &X, double value, double *x, void *stream) {
  hipLaunchKernelGGL(sfill_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     value, x);
}

void vec_select(const VecCtx &X, const double *flag, const double *src, double *dst, void *stream) {
  hipLaunchKernelGGL(sselect_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     flag, src, dst);
}

}  // namespace dmrg
