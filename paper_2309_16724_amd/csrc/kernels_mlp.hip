// Learned Davidson preconditioner: forward, backward and Adam kernels of the
// 3-layer perceptron g = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 (FP32
// storage; reductions of the backward pass accumulate in FP64 in a fixed
// order, so every result is reproducible bit for bit).
#include <hip/hip_runtime.h>
#include <cmath>
#include "mlp.hpp"

namespace dmrg {

namespace {

constexpr int MR = 64;      // rows per forward block
constexpr int NT = 256;     // threads per block

struct POff {
  int64_t W1, b1, W2, b2, w3, b3;
};
__host__ __device__ inline POff poff(int W) {
  POff o;
  o.W1 = 0;
  o.b1 = (int64_t)MLP_IN * W;
  o.W2 = o.b1 + W;
  o.b2 = o.W2 + (int64_t)W * W;
  o.w3 = o.b2 + W;
  o.b3 = o.w3 + W;
  return o;
}

__device__ inline double floored(double den, double fl) {
  return fabs(den) < fl ? (den < 0.0 ? -fl : fl) : den;
}

__device__ inline int seg_of(const int64_t *off, int nseg, int64_t i) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// MODE 0: rows from x[n][2] (optionally gathered), g out, optional activations.
// MODE 1: rows from Davidson vectors; t[i] = td_i (1 + g_i), td = -r/(d - theta).
template <int W, int MODE>
__global__ void __launch_bounds__(NT) mlp_fwd_kernel(const FwdArgs A) {
  constexpr int CPT = W / 16;          // columns per thread
  constexpr int KC = W < 32 ? W : 32;  // W2 rows per LDS chunk
  __shared__ float xs[MR][MLP_IN];
  __shared__ float h1[MR][W + 1];
  __shared__ float w2c[KC][W];
  __shared__ double tds[MR];
  const POff o = poff(W);
  const float *__restrict__ p = A.params;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * MR;
  if (tid < MR) {
    const int64_t i = row0 + tid;
    float f0 = 0.0f, f1 = 0.0f;
    double td = 0.0;
    if (i < A.n) {
      if (MODE == 0) {
        f0 = A.x[i * MLP_IN];
        f1 = A.x[i * MLP_IN + 1];
      } else {
        const int s = seg_of(A.seg_off, A.nseg, i);
        const double den = A.d[i] - A.theta[s];
        td = -A.r[i] / floored(den, A.floor_);
        f0 = (float)asinh(den / A.sigma[s]);
        f1 = (float)A.f1[s];
      }
    }
    xs[tid][0] = f0;
    xs[tid][1] = f1;
    tds[tid] = td;
  }
  __syncthreads();
  // layer 1
  for (int c = tid; c < W; c += NT) {
    const float w0 = p[o.W1 + c], w1 = p[o.W1 + W + c], bb = p[o.b1 + c];
    for (int r = 0; r < MR; r++) {
      const float z = bb + xs[r][0] * w0 + xs[r][1] * w1;
      if (A.z1 && row0 + r < A.n) A.z1[(row0 + r) * W + c] = z;
      h1[r][c] = fmaxf(z, 0.0f);
    }
  }
  // layer 2: thread (tx, ty) owns rows 4ty..4ty+3, columns tx + 16j
  float acc[4][CPT];
#pragma unroll
  for (int j = 0; j < CPT; j++) {
    const float bj = p[o.b2 + tx + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; i++) acc[i][j] = bj;
  }
  for (int k0 = 0; k0 < W; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < KC * W; e += NT) w2c[e / W][e % W] = p[o.W2 + (int64_t)(k0 + e / W) * W + e % W];
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; kk++) {
      float a[4], b[CPT];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = h1[ty * 4 + i][k0 + kk];
#pragma unroll
      for (int j = 0; j < CPT; j++) b[j] = w2c[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < CPT; j++) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
  }
  // layer 3
  float part[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    part[i] = 0.0f;
    const int64_t row = row0 + ty * 4 + i;
#pragma unroll
    for (int j = 0; j < CPT; j++) {
      const int c = tx + 16 * j;
      if (A.z2 && row < A.n) A.z2[row * W + c] = acc[i][j];
      part[i] = fmaf(fmaxf(acc[i][j], 0.0f), p[o.w3 + c], part[i]);
    }
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) part[i] += __shfl_xor(part[i], m, 16);
  }
  if (tx == 0) {
    const float b3 = p[o.b3];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int64_t row = row0 + ty * 4 + i;
      if (row >= A.n) continue;
      const float g = part[i] + b3;
      if (MODE == 0) A.g[row] = g;
      else A.t[row] = tds[ty * 4 + i] * (1.0 + (double)g);
    }
  }
}

// dg_i = 2 e_i a_i / n, e_i = a_i (1 + g_i) - b_i; per-block partial sums of e^2
__global__ void __launch_bounds__(NT) out_grad_kernel(const float *__restrict__ g, const float *__restrict__ a,
                                                      const float *__restrict__ b, int64_t n,
                                                      float *__restrict__ dg, double *__restrict__ lpart) {
  __shared__ double red[NT];
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const float e = a[i] * (1.0f + g[i]) - b[i];
    dg[i] = 2.0f * e * a[i] / (float)n;
    e2 = (double)e * (double)e;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// dz2[i][c] = dg_i w3[c] [z2[i][c] > 0]
__global__ void __launch_bounds__(NT) dz2_kernel(const float *__restrict__ dg, const float *__restrict__ z2,
                                                 const float *__restrict__ w3, int64_t n, int W,
                                                 float *__restrict__ dz2) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= n * W) return;
  const int64_t i = e / W;
  const int c = (int)(e % W);
  dz2[e] = z2[e] > 0.0f ? dg[i] * w3[c] : 0.0f;
}

// out[m][j] = sum_i Aop(i, m) Bop(i, j), FP64 accumulation in row order.
// A == nullptr: Aop = 1.  reluA/reluB: operand taken through relu.
__global__ void __launch_bounds__(NT) tn_kernel(const float *__restrict__ A, int64_t lda, int reluA,
                                                const float *__restrict__ B, int64_t ldb, int reluB, int64_t n,
                                                int M, int N, float *__restrict__ out) {
  __shared__ float As[32][33], Bs[32][33];
  const int tid = threadIdx.x, tj = tid & 31, tm = tid >> 5;   // 8 row groups x 32 columns
  const int m0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = 0; i0 < n; i0 += 32) {
    __syncthreads();
    for (int e = tid; e < 32 * 32; e += NT) {
      const int ii = e >> 5, cc = e & 31;
      const int64_t i = i0 + ii;
      float av = 0.0f, bv = 0.0f;
      if (i < n) {
        if (m0 + cc < M) {
          av = A ? A[i * lda + m0 + cc] : 1.0f;
          if (reluA) av = fmaxf(av, 0.0f);
        }
        if (j0 + cc < N) {
          bv = B[i * ldb + j0 + cc];
          if (reluB) bv = fmaxf(bv, 0.0f);
        }
      }
      As[ii][cc] = av;
      Bs[ii][cc] = bv;
    }
    __syncthreads();
    for (int ii = 0; ii < 32; ii++) {
      const double bv = Bs[ii][tj];
#pragma unroll
      for (int q = 0; q < 4; q++) acc[q] += (double)As[ii][tm + 8 * q] * bv;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int m = m0 + tm + 8 * q, j = j0 + tj;
    if (m < M && j < N) out[(int64_t)m * N + j] = (float)acc[q];
  }
}

// dz1[i][k] = (sum_j dz2[i][j] W2[k][j]) [z1[i][k] > 0], FP64 accumulation
__global__ void __launch_bounds__(NT) nt_mask_kernel(const float *__restrict__ dz2, const float *__restrict__ W2,
                                                     const float *__restrict__ z1, int64_t n, int W,
                                                     float *__restrict__ dz1) {
  __shared__ float As[32][33], Bs[32][33];
  const int tid = threadIdx.x, tk = tid & 31, ti = tid >> 5;
  const int64_t i0 = (int64_t)blockIdx.y * 32;
  const int k0 = blockIdx.x * 32;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < W; j0 += 32) {
    __syncthreads();
    for (int e = tid; e < 32 * 32; e += NT) {
      const int rr = e >> 5, cc = e & 31;
      As[rr][cc] = (i0 + rr < n) ? dz2[(i0 + rr) * W + j0 + cc] : 0.0f;
      Bs[rr][cc] = W2[(int64_t)(k0 + rr) * W + j0 + cc];
    }
    __syncthreads();
    for (int jj = 0; jj < 32; jj++) {
      const double bv = Bs[tk][jj];
#pragma unroll
      for (int q = 0; q < 4; q++) acc[q] += (double)As[ti + 8 * q][jj] * bv;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int64_t i = i0 + ti + 8 * q;
    const int k = k0 + tk;
    if (i < n) dz1[i * W + k] = z1[i * W + k] > 0.0f ? (float)acc[q] : 0.0f;
  }
}

// p -= lr mhat / (sqrt(vhat) + eps), mhat = m c1, vhat = v c2
__global__ void __launch_bounds__(NT) adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                                  const float *__restrict__ gr, int64_t n, float lr, float b1,
                                                  float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based index generator
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// minibatch gather: row j of the batch is sample splitmix64(seed + step * 2^32 + j) mod n
__global__ void __launch_bounds__(NT) gather_kernel(const float *__restrict__ x, const float *__restrict__ a,
                                                    const float *__restrict__ b, int64_t n, uint64_t seed,
                                                    uint64_t step, int batch, float *__restrict__ xb,
                                                    float *__restrict__ ab, float *__restrict__ bb) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= batch) return;
  const int64_t i = (int64_t)(splitmix64(seed + (step << 32) + (uint64_t)j) % (uint64_t)n);
  xb[j * MLP_IN] = x[i * MLP_IN];
  xb[j * MLP_IN + 1] = x[i * MLP_IN + 1];
  ab[j] = a[i];
  bb[j] = b[i];
}

// training rows of one recorded iteration: ts = psi* c - u (c = 1/<u|psi*>),
// x = (asinh((d - theta)/sigma), f1), a = td s, b = ts s, s = sqrt(n)/||ts||,
// both scaled by MLP_A_MAX/|a| where |a| exceeds MLP_A_MAX
__global__ void __launch_bounds__(NT) collect_kernel(const double *__restrict__ d, const double *__restrict__ r,
                                                     const double *__restrict__ ts, int64_t n, double theta,
                                                     double sigma, double f1, double s, double floor_,
                                                     float *__restrict__ x, float *__restrict__ a,
                                                     float *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double den = d[i] - theta;
  x[i * MLP_IN] = (float)asinh(den / sigma);
  x[i * MLP_IN + 1] = (float)f1;
  const double av = -r[i] / floored(den, floor_) * s;
  const double w = fabs(av) > MLP_A_MAX ? MLP_A_MAX / fabs(av) : 1.0;
  a[i] = (float)(av * w);
  b[i] = (float)(ts[i] * s * w);
}

__global__ void __launch_bounds__(NT) exact_corr_kernel(const double *__restrict__ psi, const double *__restrict__ u,
                                                        int64_t n, double c, double *__restrict__ ts) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) ts[i] = psi[i] * c - u[i];
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + NT - 1) / NT)); }

}  // namespace

bool mlp_width_ok(int W) { return W == 32 || W == 64 || W == 128 || W == 256; }

void launch_mlp_forward(int W, int mode, const FwdArgs &A, void *stream) {
  const dim3 grid((unsigned)((A.n + MR - 1) / MR));
  hipStream_t s = (hipStream_t)stream;
#define FWD(w)                                                                                   \
  case w:                                                                                        \
    if (mode == 0) hipLaunchKernelGGL((mlp_fwd_kernel<w, 0>), grid, dim3(NT), 0, s, A);          \
    else hipLaunchKernelGGL((mlp_fwd_kernel<w, 1>), grid, dim3(NT), 0, s, A);                    \
    break;
  switch (W) { FWD(32) FWD(64) FWD(128) FWD(256) default: break; }
#undef FWD
}

void launch_mlp_backward(int W, const float *params, const float *x, const float *a, const float *b,
                         int64_t n, const float *g, const float *z1, const float *z2, float *dg, float *dz2,
                         float *dz1, double *lpart, float *grad, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const POff o = poff(W);
  hipLaunchKernelGGL(out_grad_kernel, grid1(n), dim3(NT), 0, s, g, a, b, n, dg, lpart);
  hipLaunchKernelGGL(dz2_kernel, grid1(n * W), dim3(NT), 0, s, dg, z2, params + o.w3, n, W, dz2);
  auto tn = [&](const float *A_, int64_t lda, int rA, const float *B_, int64_t ldb, int rB, int M, int N, float *out) {
    dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
    hipLaunchKernelGGL(tn_kernel, grid, dim3(NT), 0, s, A_, lda, rA, B_, ldb, rB, n, M, N, out);
  };
  tn(z1, W, 1, dz2, W, 0, W, W, grad + o.W2);          // dW2 = relu(z1)^T dz2
  tn(nullptr, 0, 0, dz2, W, 0, 1, W, grad + o.b2);     // db2
  tn(dg, 1, 0, z2, W, 1, 1, W, grad + o.w3);           // dw3 = dg^T relu(z2)
  tn(nullptr, 0, 0, dg, 1, 0, 1, 1, grad + o.b3);      // db3
  dim3 gnt((unsigned)(W / 32), (unsigned)((n + 31) / 32));
  hipLaunchKernelGGL(nt_mask_kernel, gnt, dim3(NT), 0, s, dz2, params + o.W2, z1, n, W, dz1);
  tn(x, MLP_IN, 0, dz1, W, 0, MLP_IN, W, grad + o.W1); // dW1 = x^T dz1
  tn(nullptr, 0, 0, dz1, W, 0, 1, W, grad + o.b1);     // db1
}

void launch_adam(float *p, float *m, float *v, const float *gr, int64_t n, float lr, float b1, float b2, float eps,
                 float c1, float c2, void *stream) {
  hipLaunchKernelGGL(adam_kernel, grid1(n), dim3(NT), 0, (hipStream_t)stream, p, m, v, gr, n, lr, b1, b2, eps, c1,
                     c2);
}

void launch_gather(const float *x, const float *a, const float *b, int64_t n, uint64_t seed, uint64_t step, int batch,
                   float *xb, float *ab, float *bb, void *stream) {
  hipLaunchKernelGGL(gather_kernel, grid1(batch), dim3(NT), 0, (hipStream_t)stream, x, a, b, n, seed, step, batch,
                     xb, ab, bb);
}

void launch_exact_corr(const double *psi, const double *u, int64_t n, double c, double *ts, void *stream) {
  hipLaunchKernelGGL(exact_corr_kernel, grid1(n), dim3(NT), 0, (hipStream_t)stream, psi, u, n, c, ts);
}

void launch_collect(const double *d, const double *r, const double *ts, int64_t n, double theta, double sigma,
                    double f1, double s, double floor_, float *x, float *a, float *b, void *stream) {
  hipLaunchKernelGGL(collect_kernel, grid1(n), dim3(NT), 0, (hipStream_t)stream, d, r, ts, n, theta, sigma, f1, s,
                     floor_, x, a, b);
}

}  // namespace dmrg
