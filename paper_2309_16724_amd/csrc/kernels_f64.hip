// FP64 MFMA kernels for the grouped stripe products of H.psi.
//
// Every H.psi is two launches of the same tile kernel: the first computes
// T = X op(D) for each wavefunction block and right-block operator and
// writes it as a vertical stripe over positions; the second accumulates
// Y_F += v A_stripe T_stripe for every output block F (output stationary: a
// tile owns its outputs, no atomics).  One wavefront computes a 32x32 tile
// as 2x2 v_mfma_f64_16x16x4 products, operands staged through LDS.
// Lane layout of v_mfma_f64_16x16x4f64 (lane l, accumulator element r):
// A[l%16][l/16], B[l/16][l%16], D[l/16 + 4r][l%16].
#include <hip/hip_runtime.h>
#include "plan.hpp"

namespace dmrg {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ const double *base_ptr(int id, const double *const *bases, const double *psi,
                                                  const double *y, const double *work) {
  return id == BASE_PSI ? psi : id == BASE_Y ? y : id == BASE_WORK ? work : bases[id - BASE_OPS];
}

__device__ __forceinline__ void tiles_f64(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,
                                          int ntiles, const double *const *__restrict__ bases,
                                          const double *__restrict__ psi, double *__restrict__ y,
                                          double *__restrict__ work) {
  __shared__ double As[TILE][17];
  __shared__ double Bs[16][TILE + 1];
  const int lane = threadIdx.x;
  const int r16 = lane & 15, q4 = lane >> 4;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile T = tiles[t];
    v4d acc[2][2];
    for (int a = 0; a < 2; a++)
      for (int b = 0; b < 2; b++) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    const int mrem = T.m - T.i0, nrem = T.n - T.j0;
    for (int si = 0; si < T.nseg; si++) {
      const Seg S = segs[T.seg0 + si];
      const double *B = base_ptr(S.b_base, bases, psi, y, work) + S.b_off;
      if (S.a_base < 0) {
        // identity left operator: tile += s * B (B has the tile's row count)
        for (int bi = 0; bi < 2; bi++)
          for (int bj = 0; bj < 2; bj++)
            for (int r = 0; r < 4; r++) {
              int i = 16 * bi + q4 + 4 * r, j = 16 * bj + r16;
              if (i < mrem && j < nrem)
                acc[bi][bj][r] += S.s * B[(int64_t)(T.i0 + i) * S.b_k + (int64_t)(T.j0 + j) * S.b_j];
            }
        continue;
      }
      const double *A = base_ptr(S.a_base, bases, psi, y, work) + S.a_off;
      for (int k0 = 0; k0 < S.K; k0 += 16) {
        for (int e = lane; e < TILE * 16; e += 64) {
          int i = e & (TILE - 1), kk = e / TILE;
          int gi = T.i0 + i, gk = k0 + kk;
          double v = 0.0;
          if (i < mrem && gk < S.K) {
            int p = gk / S.kb, kr = gk - p * S.kb;
            v = S.s * A[(int64_t)p * S.a_p + (int64_t)gi * S.a_i + (int64_t)kr * S.a_k];
          }
          As[i][kk] = v;
        }
        for (int e = lane; e < TILE * 16; e += 64) {
          int kk = e & 15, j = e >> 4;
          int gk = k0 + kk, gj = T.j0 + j;
          double v = 0.0;
          if (j < nrem && gk < S.K) v = B[(int64_t)gk * S.b_k + (int64_t)gj * S.b_j];
          Bs[kk][j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
          double a0 = As[r16][kk + q4], a1 = As[r16 + 16][kk + q4];
          double b0 = Bs[kk + q4][r16], b1 = Bs[kk + q4][r16 + 16];
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
      }
    }
    double *C = const_cast<double *>(base_ptr(T.c_base, bases, psi, y, work)) + T.c_off;
    for (int bi = 0; bi < 2; bi++)
      for (int bj = 0; bj < 2; bj++)
        for (int r = 0; r < 4; r++) {
          int i = 16 * bi + q4 + 4 * r, j = 16 * bj + r16;
          if (i < mrem && j < nrem) {
            double *c = C + (int64_t)(T.i0 + i) + (int64_t)(T.j0 + j) * T.ldc;
            *c = T.accumulate ? *c + acc[bi][bj][r] : acc[bi][bj][r];
          }
        }
  }
}

// first stage: T stripes = X op(D)
__global__ void __launch_bounds__(64) stage1_f64_kernel(const Tile *__restrict__ tiles,
                                                         const Seg *__restrict__ segs, int ntiles,
                                                         const double *const *__restrict__ bases,
                                                         const double *__restrict__ psi,
                                                         double *__restrict__ y, double *__restrict__ work) {
  tiles_f64(tiles, segs, ntiles, bases, psi, y, work);
}

// second stage: Y_F += sum v A_stripe T_stripe (output stationary)
__global__ void __launch_bounds__(64) stage2_f64_kernel(const Tile *__restrict__ tiles,
                                                         const Seg *__restrict__ segs, int ntiles,
                                                         const double *const *__restrict__ bases,
                                                         const double *__restrict__ psi,
                                                         double *__restrict__ y, double *__restrict__ work) {
  tiles_f64(tiles, segs, ntiles, bases, psi, y, work);
}

__global__ void zero_kernel(double *y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = 0.0;
}

__global__ void diag_kernel(const DiagBlock *__restrict__ blocks, const DiagTerm *__restrict__ terms,
                            int nblocks, const double *const *__restrict__ bases, double *__restrict__ diag) {
  for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const DiagBlock B = blocks[b];
    int64_t n = (int64_t)B.m * B.n;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
      int i = (int)(e % B.m), j = (int)(e / B.m);
      double acc = 0.0;
      for (int t = 0; t < B.nt; t++) {
        const DiagTerm T = terms[B.t0 + t];
        double a = T.a_base < 0 ? 1.0 : bases[T.a_base - BASE_OPS][T.a_off + (int64_t)i * T.a_step];
        double d = T.d_base < 0 ? 1.0 : bases[T.d_base - BASE_OPS][T.d_off + (int64_t)j * T.d_step];
        acc += T.s * a * d;
      }
      diag[B.off + e] = acc;
    }
  }
}

void launch_zero(double *y, int64_t n, void *stream) {
  if (n <= 0) return;
  int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, y, n);
}

void launch_tiles_f64(int stage, const Tile *tiles, const Seg *segs, int ntiles, const double *const *bases,
                      const double *psi, double *y, double *work, void *stream) {
  if (ntiles <= 0) return;
  int grid = std::min(ntiles, 256 * 16);
  if (stage == 1)
    hipLaunchKernelGGL(stage1_f64_kernel, dim3(grid), dim3(64), 0, (hipStream_t)stream, tiles, segs,
                       ntiles, bases, psi, y, work);
  else
    hipLaunchKernelGGL(stage2_f64_kernel, dim3(grid), dim3(64), 0, (hipStream_t)stream, tiles, segs,
                       ntiles, bases, psi, y, work);
}

void launch_diag(const DiagBlock *blocks, const DiagTerm *terms, int nblocks, const double *const *bases,
                 double *diag, void *stream) {
  if (nblocks <= 0) return;
  int grid = std::min(nblocks, 4096);
  hipLaunchKernelGGL(diag_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, blocks, terms, nblocks,
                     bases, diag);
}

}  // namespace dmrg
