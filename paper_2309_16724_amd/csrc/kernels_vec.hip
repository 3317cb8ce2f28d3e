// FP64 vector kernels of the Davidson solver.  Vectors are concatenations of
// one segment per problem; work is cut into chunks that never cross a
// segment, and every reduction is two-pass (per-chunk partial sums, then a
// fixed-order sum per segment), so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include "davidson.hpp"

namespace dmrg {

constexpr int VB = 256;          // threads per block

// part[c * m + j] = sum_{i in chunk c} V[j * ldv + i] * x[i], j < m
static_assert(VCHUNK % VB == 0 && VCHUNK / VB <= 8, "a thread holds VCHUNK / VB elements of x");
// part[c * m + j] = sum over chunk c of V[j * ldv + i] x[i]: x stays in
// registers, each column is reduced within the wavefront by shuffles, and the
// four wavefronts' partials are added in wave order after one barrier (fixed
// order throughout: reproducible bit for bit).
__global__ void __launch_bounds__(VB) sdots_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                    const double *__restrict__ V, int64_t ldv, int m,
                                                    const double *__restrict__ x, double *__restrict__ part) {
  constexpr int PT = VCHUNK / VB, NW = VB / 64;
  __shared__ double red[NW][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    double xv[PT];
    int64_t idx[PT];
#pragma unroll
    for (int e = 0; e < PT; e++) {
      idx[e] = C.i0 + threadIdx.x + (int64_t)e * VB;
      xv[e] = idx[e] < C.i1 ? x[idx[e]] : 0.0;
    }
    for (int j0 = 0; j0 < m; j0 += 64) {
      const int jn = min(64, m - j0);
      for (int jj = 0; jj < jn; jj++) {
        const double *v = V + (int64_t)(j0 + jj) * ldv;
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < PT; e++)
          if (idx[e] < C.i1) acc += v[idx[e]] * xv[e];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) red[wave][jj] = acc;
      }
      __syncthreads();
      if ((int)threadIdx.x < jn) {
        double s = 0.0;
        for (int w = 0; w < NW; w++) s += red[w][threadIdx.x];
        part[(int64_t)c * m + j0 + threadIdx.x] = s;
      }
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
      // four columns per round: independent loads in flight, fixed order
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int j = 0;
      for (; j + 3 < m; j += 4) {
        a0 += cf[j] * V[(int64_t)j * ldv + i];
        a1 += cf[j + 1] * V[(int64_t)(j + 1) * ldv + i];
        a2 += cf[j + 2] * V[(int64_t)(j + 2) * ldv + i];
        a3 += cf[j + 3] * V[(int64_t)(j + 3) * ldv + i];
      }
      for (; j < m; j++) a0 += cf[j] * V[(int64_t)j * ldv + i];
      const double acc = (a0 + a1) + (a2 + a3);
      y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + sign * acc;
    }
  }
}

// r = hu - theta_k u ; t = -r / (diag - theta_k) with |denominator| >= floor_k
// (per-segment absolute floors)
__global__ void __launch_bounds__(VB) sresid_kernel(const VChunk *__restrict__ chunks, int nchunks,
                                                     const double *__restrict__ hu, const double *__restrict__ u,
                                                     const double *__restrict__ diag,
                                                     const double *__restrict__ theta,
                                                     const double *__restrict__ floors,
                                                     double *__restrict__ r, double *__restrict__ t) {
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const VChunk C = chunks[c];
    const double th = theta[C.seg], floor_ = floors[C.seg];
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
               const double *floors, double *r, double *t, void *stream) {
  hipLaunchKernelGGL(sresid_kernel, dim3(cgrid(X.nchunks)), dim3(VB), 0, (hipStream_t)stream, X.chunks, X.nchunks,
                     hu, u, diag, theta, floors, r, t);
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
