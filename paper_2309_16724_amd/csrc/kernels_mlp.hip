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

typedef float v4f __attribute__((ext_vector_type(4)));

// Output row (within a wavefront's 16) of accumulator element r held by lane
// group q = lane / 16 in v_mfma_f32_16x16x4f32; the column is lane % 16.
// Operands: A[lane % 16][lane / 16], B[lane / 16][lane % 16].
__device__ constexpr int mfma_row(int q, int r) { return 4 * q + r; }

// Features (x0, x1) and, in MODE 1, the diagonal step td of row i.
template <int MODE>
__device__ inline void row_inputs(const FwdArgs &A, int64_t i, float &f0, float &f1, double &td) {
  f0 = f1 = 0.0f;
  td = 0.0;
  if (i >= A.n) return;
  if (MODE == 0) {
    f0 = A.x[i * MLP_IN];
    f1 = A.x[i * MLP_IN + 1];
  } else {
    const int s = seg_of(A.seg_off, A.nseg, i);
    const double den = A.d[i] - A.theta[s];
    td = -A.r[i] / floored(den, A.floor_[s]);
    f0 = (float)asinh(den / A.sigma[s]);
    f1 = (float)A.f1[s];
  }
}

// MODE 0: rows from x[n][2], g out, optional activations z1, z2 (training).
// MODE 1: rows from Davidson vectors; t[i] = td_i (1 + g_i), td = -r/(d - theta).
// Each wavefront takes 16 rows.  Layer 1 goes straight into registers: lane
// l holds relu(z1) of row l % 16 at k = 4j + l / 16, j < W/4 -- exactly the A
// operand of the K steps of layer 2, which runs on v_mfma_f32_16x16x4f32 over
// W/16 column blocks with W2 staged through LDS in chunks of 32 rows shared
// by the work group's four wavefronts.  Layer 3 reduces over the 16 lanes of
// each output row.
template <int W, int MODE>
__global__ void __launch_bounds__(NT) mlp_fwd_kernel(const FwdArgs A) {
  static_assert(W % 32 == 0 && MR == 64 && NT == 256, "64 rows of 4 wavefronts, W2 chunks of 32 rows");
  constexpr int NB = W / 16, KS = W / 4, KC = 32;
  __shared__ float w2c[KC][W];
  const POff o = poff(W);
  const float *__restrict__ p = A.params;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * MR + wave * 16;
  const int64_t arow = base + l16;
  float f0, f1;
  double td_unused;
  row_inputs<MODE>(A, arow, f0, f1, td_unused);
  float h[KS];
#pragma unroll
  for (int j = 0; j < KS; j++) {
    const int k = 4 * j + q;
    const float z = p[o.b1 + k] + f0 * p[o.W1 + k] + f1 * p[o.W1 + W + k];
    if (MODE == 0 && A.z1 && arow < A.n) A.z1[arow * W + k] = z;
    h[j] = fmaxf(z, 0.0f);
  }
  v4f acc[NB];
#pragma unroll
  for (int bj = 0; bj < NB; bj++) acc[bj] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < W; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < KC * W; e += NT) w2c[e / W][e % W] = p[o.W2 + (int64_t)(k0 + e / W) * W + e % W];
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const float a = h[(k0 + kk) / 4];
#pragma unroll
      for (int bj = 0; bj < NB; bj++)
        acc[bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w2c[kk + q][16 * bj + l16], acc[bj], 0, 0, 0);
    }
  }
  // layer 3
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int bj = 0; bj < NB; bj++) {
    const int c = 16 * bj + l16;
    const float bb = p[o.b2 + c], w3 = p[o.w3 + c];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const float z = acc[bj][r] + bb;
      const int64_t orow = base + mfma_row(q, r);
      if (MODE == 0 && A.z2 && orow < A.n) A.z2[orow * W + c] = z;
      part[r] = fmaf(fmaxf(z, 0.0f), w3, part[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; r++)
    for (int m = 8; m > 0; m >>= 1) part[r] += __shfl_xor(part[r], m, 16);
  if (l16 == 0) {
    const float b3 = p[o.b3];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int64_t orow = base + mfma_row(q, r);
      if (orow >= A.n) continue;
      const float g = part[r] + b3;
      if (MODE == 0) {
        A.g[orow] = g;
      } else {
        float x0, x1;
        double td;
        row_inputs<1>(A, orow, x0, x1, td);
        A.t[orow] = td * (1.0 + (double)g);
      }
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
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
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
