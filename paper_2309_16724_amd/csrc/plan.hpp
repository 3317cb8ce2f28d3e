// Device plan: stripe products (Sec. III A) as grouped GEMM tiles.
#pragma once
#include "common.hpp"

namespace dmrg {

// Operand bases: 0 = psi (input), 1 = hpsi (output), 2 = stripe workspace,
// 3 + k = operator data array k (left/right data of every problem).
enum { BASE_PSI = 0, BASE_Y = 1, BASE_WORK = 2, BASE_OPS = 3 };

// One stripe product contributing to a tile: tile += s * op(A)[rows, 0:K] * B[0:K, cols]
//   A(i, k) = A[(k / kb) * a_p + i * a_i + (k % kb) * a_k]   (a_base < 0: identity A)
//   B(k, j) = B[k * b_k + j * b_j]
struct Seg {
  int64_t a_off, b_off;
  int64_t a_p, a_i, a_k;
  int64_t b_k, b_j;
  double s;
  int32_t a_base, b_base;
  int32_t K, kb;
};

// One output tile of TILE x TILE elements of an m x n column-major block.
struct Tile {
  int64_t c_off;
  int64_t ldc;
  int32_t c_base;
  int32_t m, n, i0, j0;
  int32_t seg0, nseg;
  int32_t accumulate;   // 1: C += acc, 0: C = acc
};

// Diagonal of H_eff: diag[off + i + j*m] += s * dA_i * dD_j over a block's list
struct DiagTerm {
  int64_t a_off, d_off;       // diagonal element base offsets
  int64_t a_step, d_step;     // stride between consecutive diagonal elements
  double s;
  int32_t a_base, d_base;     // -1: identity
};
struct DiagBlock {
  int64_t off;
  int32_t m, n;
  int32_t t0, nt;
};

struct Chunk {
  std::vector<Seg> seg1, seg2;
  std::vector<Tile> tile1, tile2;
  Seg *d_seg1 = nullptr, *d_seg2 = nullptr;
  Tile *d_tile1 = nullptr, *d_tile2 = nullptr;
  double flops1 = 0.0, flops2 = 0.0;    // algorithmic flops of each launch
};

constexpr int TILE = 32;

void launch_zero(double *y, int64_t n, void *stream);
void launch_tiles_f64(int stage, const Tile *tiles, const Seg *segs, int ntiles, const double *const *bases,
                      const double *psi, double *y, double *work, void *stream);
void launch_diag(const DiagBlock *blocks, const DiagTerm *terms, int nblocks,
                 const double *const *bases, double *diag, void *stream);

}  // namespace dmrg
