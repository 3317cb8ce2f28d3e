// Device plan: stripe products (Sec. III A) as grouped GEMM tiles.
#pragma once
#include "common.hpp"

namespace dmrg {

// Operand bases: 0 = psi (input), 1 = hpsi (output), 2 = stripe workspace,
// 3 = partial-tile buffer, 4 + k = operator data array k.
enum { BASE_PSI = 0, BASE_Y = 1, BASE_WORK = 2, BASE_PART = 3, BASE_OPS = 4 };

// One stripe product contributing to a tile: tile += s * op(A)[rows, 0:K] * B[0:K, cols].
// Operands are stacks of blocks along K (positions) and, for B, along N:
//   A(i, k) = A[(k / a_kb) * a_p + i * a_i + (k % a_kb) * a_k]      (a_base < 0: identity)
//   B(k, n) = B[(k / b_kb) * b_pk + (k % b_kb) * b_k + (n / b_nb) * b_pn + (n % b_nb) * b_n]
struct Seg {
  int64_t a_off, b_off;
  int64_t a_p, a_i, a_k;
  int64_t b_pk, b_k, b_pn, b_n;
  double s;
  int32_t a_base, b_base;
  int32_t K, a_kb, b_kb, b_nb;
};

// One work item: a (16*mb) x (64/mb) tile of an m x n column-major output
// block (rows i0.., columns j0..) accumulated over segments seg0..seg0+nseg-1
// and stored at C + (ci0 + i) + (cj0 + j) * ldc (C += or C =).
struct Tile {
  int64_t c_off;
  int64_t ldc;
  int32_t c_base;
  int32_t m, n, i0, j0;
  int32_t ci0, cj0;
  int32_t mb;           // MFMA row blocks: 1, 2 or 4 (column blocks 4 / mb)
  int32_t seg0, nseg;
  int32_t accumulate;   // 1: C += acc, 0: C = acc
};

// Deterministic sum of the partial tiles of one output tile into Y.
struct Reduce {
  int64_t y_off, ldc;
  int64_t part_off;     // first partial; partial p at part_off + p * 1024
  int32_t m, n, i0, j0, tm, nparts;
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

// One dressed position: dst[0:n] = sum_t alpha[t] * src[src_off[t] + 0:n]
struct DressItem {
  int64_t dst_off, n;
  int32_t t0, t1;
  int32_t src_base, dst_base;
};

struct Chunk {
  std::vector<Seg> seg1, seg2;
  std::vector<Tile> tile1, tile2;
  std::vector<Reduce> red2;
  Seg *d_seg1 = nullptr, *d_seg2 = nullptr;
  Tile *d_tile1 = nullptr, *d_tile2 = nullptr;
  Reduce *d_red2 = nullptr;
  double flops1 = 0.0, flops2 = 0.0;    // algorithmic flops of each launch
  int64_t part_elems = 0;               // partial-tile buffer needed
};

constexpr int TILE = 32;      // nominal tile edge (tiles are 16*mb x 64/mb)
constexpr int WAVES = 4;      // wavefronts per workgroup (one work item each)
constexpr int KPART = 2048;   // target summed K of one second-stage work item

void launch_zero(double *y, int64_t n, void *stream);
void launch_dress(const DressItem *items, int nitems, const int64_t *src_off, const double *alpha,
                  const double *const *bases, double *dst, void *stream);
void launch_tiles_f64(int stage, const Tile *tiles, const Seg *segs, int ntiles, const double *const *bases,
                      const double *psi, double *y, double *work, double *part, void *stream);
void launch_reduce(const Reduce *red, int nred, const double *part, double *y, void *stream);
void launch_diag(const DiagBlock *blocks, const DiagTerm *terms, int nblocks,
                 const double *const *bases, double *diag, void *stream);

}  // namespace dmrg
