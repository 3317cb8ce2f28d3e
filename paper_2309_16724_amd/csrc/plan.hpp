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

// Work-group tiles: a tile with mb == MACRO_MB is a 64 x 64 tile computed by
// the four wavefronts of a work group together (each a 32 x 32 quarter) from
// operand tiles they stage in LDS once; the other tiles belong to one
// wavefront each.
constexpr int MACRO_MB = 8;
constexpr int MACRO_EDGE = 64;
constexpr int MACRO_MIN = 48;   // default: outputs with both dims >= 48 get work-group tiles
// Wide work-group tiles (split plans, s <= 5): WIDE_MB tiles are 128 x 128,
// computed by the eight wavefronts of a work group (two per SIMD, 32 x 64
// each, v_mfma_f32_32x32x16_bf16) from two 80 KiB LDS stages.  An
// output with both sides >= wide_min is cut into 128-wide bands (a last band
// of >= wide_min lines is a wide band too); the rest of it gets 64 x 64 or
// wavefront tiles.
constexpr int WIDE_MB = 16;
constexpr int WIDE_EDGE = 128;
constexpr int WIDE_MIN = 48;
constexpr int WIDE_WAVES = 8;
constexpr int WIDE_MAX_SLICES = 5;
constexpr int tile_rows(int mb) { return mb == WIDE_MB ? WIDE_EDGE : mb == MACRO_MB ? MACRO_EDGE : 16 * mb; }
constexpr int tile_cols(int mb) { return mb == WIDE_MB ? WIDE_EDGE : mb == MACRO_MB ? MACRO_EDGE : 64 / mb; }

// Per-XCD queues of a work-group tile list: the list (cost-sorted, operand
// bands in patches) is cut into NXCD contiguous ranges of equal cost; the work
// groups of XCD x take the tiles of range x in order through an atomic
// counter and then help the other ranges, so the tiles that run side by side
// on one XCD are neighbours in the list and share operand bands in its L2.
constexpr int NXCD = 8;
constexpr int MACRO_GRID = 512;          // work groups of a work-group tile launch (two per CU)
constexpr int WIDE_GRID = 256;           // work groups of a wide tile launch (one per CU)
constexpr int QUEUE_INTS = NXCD + MACRO_GRID;   // queue counters, then one mailbox per work group
struct XcdQueues {
  int32_t start[NXCD + 1];
};

// One work item: a (16*mb) x (64/mb) tile of an m x n output block (rows
// i0.., columns j0..) accumulated over segments seg0..seg0+nseg-1 and stored
// at C + (ci0 + i) + (cj0 + j) * ldc (column-major) or at
// C + (ci0 + i) * ldc + (cj0 + j) (rowmajor) (C += or C =).
struct Tile {
  int64_t c_off;
  int64_t ldc;
  int32_t c_base;
  int32_t m, n, i0, j0;
  int32_t ci0, cj0;
  int32_t mb;           // MFMA row blocks: 1, 2 or 4 (column blocks 4 / mb)
  int32_t seg0, nseg;
  int32_t accumulate;   // 1: C += acc, 0: C = acc
  int32_t rowmajor;     // output layout, see above
};

// Transposed copy of one operator record: npos column-major rows x cols
// blocks at off become cols x rows blocks at the same offset.
struct TransJob {
  int64_t off;
  int32_t rows, cols, npos, pad;
};

// Deterministic sum of the partial tiles of one output tile into Y.
struct Reduce {
  int64_t y_off, ldc;
  int64_t part_off;     // first partial; partial p at part_off + p * tm * tn (column-major, ld tm)
  int32_t m, n, i0, j0, tm, tn, nparts, pad;
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

// ---------------------------------------------------------------- split BF16
// Fixed-point slicing (Ozaki-style): a line x (row of an A operand or column
// of a B operand, over its K range) is scaled by 2^-e with e the smallest
// integer such that max|x| <= 2^e, then cut into s integer digits of SLICE_BITS
// bits, x = 2^e sum_t a_t 2^(-8(t+1)) + O(2^(e-8s)), |a_0| <= 256, |a_t| <= 128.
// Slice t stores a_t 2^(-8t), exact in BF16 (at most 8 significant bits), so
// that a product of slices t and u already carries the relative weight
// 2^(-8(t+u)) of its group d = t + u and every group folds with 2^-16.  Lines
// are stored K-contiguous (operand-ready), each position block of K padded to
// a multiple of 8 with zeros, and the s slices interleaved per chunk of 8: the
// element at index e of the unsliced layout (offsets, line lengths: multiples
// of 8) has slice t at (e - e % 8) s + 8 t + e % 8 (slice_index), so that the
// s slices of a K step of a line are one contiguous run of memory.
constexpr int SLICE_BITS = 8;
// Slice products accumulate in slice_groups(s) FP32 sums: groups d = t + u
// below s - 3 each in its own sum, exact, and all groups d >= s - 3 in one
// more sum (for s <= 3 that is the only one).  Per k an exact group d is at
// most 2^16 (d <= 1) or (d + 3) 2^14 (d >= 2) in units of its resolution
// 2^(-8d), so over split_fold_k(s) terms its sum stays an integer (in those
// units) below 2^24: exact in FP32.  The merged sum is rounded, but its terms
// weigh at most about 2^(-8(s-3)+1) of group 0, so FP32 rounding (2^-24) puts
// its error at the level of the truncation after s digits (2^-8s).  Every
// split_fold_k(s) terms of K the sums are folded into FP64.
constexpr int slice_groups(int ns) { return ns <= 3 ? 1 : ns - 2; }
constexpr int split_fold_k(int ns) { return ns <= 5 ? 256 : 128; }

// One slicing job: lines rho < nrho, position blocks p < npos of kb valid
// entries (padded to kbp);  source x(rho, p, kk) at src[src_off + rho*s_rho + p*s_pos + kk*s_k];
// slice t of the element at e = dst_off + rho*npos*kbp + p*kbp + kk at dst[slice_index(e, t, s)];
// exponent of line rho at exps[exp_off + rho].
struct SliceJob {
  int64_t src_off, s_rho, s_pos, s_k;
  int64_t dst_off, exp_off;
  int32_t src_base, dst_buf;
  int32_t nrho, npos, kb, kbp;
};

// Split segment (same role as Seg): A lines are operand rows, B lines operand
// columns, both K-contiguous in slice buffers.
struct SegS {
  int64_t a_off, a_ld, a_exp;
  int64_t b_off, b_ld, b_exp;
  int32_t a_buf, b_buf;
  int32_t K;          // padded K (multiple of 8); 0 for an identity segment
  int32_t t_nb;       // first-stage segments: stripe columns per slot (line = column mod t_nb)
  int64_t t_exp;      // first-stage segments: exponent offset of the stripe's lines, else -1
};

// Stripe slicing work item: elements [e0, e0 + TSLICE_CHUNK) of job `job`,
// flattened line by line (line rho, then padded index along its K range).
constexpr int TSLICE_CHUNK = 1024;
struct TSliceItem {
  int32_t job, e0;
};

// slice buffers: 0 operator records (plan), 1 psi rows, 2 psi columns, 3 stripes
enum { SBUF_OPS = 0, SBUF_PSIR = 1, SBUF_PSIC = 2, SBUF_T = 3, N_SBUF = 4 };

struct SliceBufs {
  uint16_t *data[N_SBUF];     // bf16 bit patterns, slices interleaved (slice_index)
  int32_t *exps[N_SBUF];
};
// position of slice t of element e (index in the unsliced layout) for s slices
__host__ __device__ inline int64_t slice_index(int64_t e, int t, int s) { return (e - (e & 7)) * s + 8 * t + (e & 7); }


// bookkeeping that lets the split-precision plan mirror the FP64 segments
struct StripeInfo {
  int prob, E, rec, adj, dress;
  int64_t off;
  int dL, dRin, dRout, nslots;
  int first_slot_pos;          // unused
};
struct Seg1Info { int stripe, s0, pD0; };
struct Seg2Info { int prob, E, stripe, slot0, recA, adjA, pA0, run; };

struct Chunk {
  std::vector<StripeInfo> stripes;
  std::vector<Seg1Info> s1info;
  std::vector<Seg2Info> s2info;
  std::vector<Seg> seg1, seg2;
  std::vector<Tile> tile1, tile2;       // one wavefront per tile
  std::vector<Tile> tile1m, tile2m;     // work-group (macro) tiles
  std::vector<Tile> tile1x, tile2x;     // wide work-group tiles
  XcdQueues q1{}, q2{}, q1m{}, q2m{}, q1x{}, q2x{};   // per-XCD ranges of the six lists
  std::vector<Reduce> red2;
  Seg *d_seg1 = nullptr, *d_seg2 = nullptr;
  Tile *d_tile1 = nullptr, *d_tile2 = nullptr;
  Tile *d_tile1m = nullptr, *d_tile2m = nullptr;
  Tile *d_tile1x = nullptr, *d_tile2x = nullptr;
  Reduce *d_red2 = nullptr;
  double flops1 = 0.0, flops2 = 0.0;    // algorithmic flops of each stage
  double flops1m = 0.0, flops2m = 0.0;  // ... of its work-group tiles
  double flops1x = 0.0, flops2x = 0.0;  // ... of its wide tiles
  double flops1w = 0.0, flops2w = 0.0;  // ... of its wavefront tiles
  int64_t part_elems = 0;               // partial-tile buffer needed
  // split precision (filled only for split plans)
  std::vector<SegS> sseg1, sseg2;
  std::vector<SliceJob> tjobs;          // stripe slicing after the first stage
  std::vector<TSliceItem> titems;       // its element chunks
  SegS *d_sseg1 = nullptr, *d_sseg2 = nullptr;
  SliceJob *d_tjobs = nullptr;
  TSliceItem *d_titems = nullptr;
  int64_t t_elems = 0, t_exps = 0;
};

constexpr int TILE = 32;      // nominal tile edge (tiles are 16*mb x 64/mb)
constexpr int WAVES = 4;      // wavefronts per workgroup (one work item each)
constexpr int KPART = 2048;   // target summed K of one second-stage work item
// default cap of the stripe workspace (288 GB of HBM hold the largest plans in one chunk)
constexpr int64_t DEFAULT_WORKSPACE = (int64_t)64 << 30;

void launch_zero(double *y, int64_t n, void *stream);
void launch_dress(const DressItem *items, int nitems, const int64_t *src_off, const double *alpha,
                  const double *const *bases, double *dst, void *stream);
// tiles from per-XCD queues; counters: QUEUE_INTS ints of device memory, the
// NXCD queue counters cleared by this call before the launch
void launch_tiles_f64(int stage, const Tile *tiles, const Seg *segs, int ntiles, const XcdQueues &q,
                      int32_t *counters, const double *const *bases, const double *psi, double *y, double *work,
                      double *part, void *stream);
void launch_reduce(const Reduce *red, int nred, const double *part, double *y, void *stream);
void launch_transpose(const TransJob *jobs, int njobs, const double *src, double *dst, void *stream);
void launch_diag(const DiagBlock *blocks, const DiagTerm *terms, int nblocks,
                 const double *const *bases, double *diag, void *stream);

}  // namespace dmrg

namespace dmrg {
void launch_slices(const SliceJob *jobs, int njobs, int nslices, const double *const *bases, const double *psi,
                   const double *work, SliceBufs bufs, void *stream);
// stripe slicing with line exponents already in place (the first stage's
// epilogue takes their maxima with atomicMax; sentinel INT_MIN = all zero)
void launch_tslices(const SliceJob *jobs, const TSliceItem *items, int nitems, int nslices, const double *work,
                    SliceBufs bufs, void *stream);
void launch_fill_int(int32_t *p, int64_t n, int32_t v, void *stream);
// scratch memory of one H.psi: byte offsets of the stripe workspace, partial
// tiles, stripe slices, stripe exponents and work-queue counters; returns the
// total bytes
constexpr int SCRATCH_REGIONS = 5;
int64_t plan_scratch_layout(const dmrg_plan_t *p, int64_t off[SCRATCH_REGIONS]);
// one H.psi with that scratch memory at base (device address)
int enqueue_scratch(dmrg_plan_t *p, const double *psi, double *hpsi, void *stream, char *base);
// wavefront tiles (one tile per wavefront) from per-XCD queues
void launch_tiles_split(int stage, const Tile *tiles, const Seg *segs, const SegS *ssegs, int ntiles,
                        const XcdQueues &q, int32_t *counters, int nslices, const double *const *bases,
                        const double *psi, double *y, double *work, double *part, SliceBufs bufs, void *stream);
// work-group (MACRO_MB) tiles from per-XCD queues; counters: QUEUE_INTS ints
// of device memory, the NXCD queue counters cleared by this call before the launch
void launch_macro_split(int stage, const Tile *tiles, const Seg *segs, const SegS *ssegs, int ntiles,
                        const XcdQueues &q, int32_t *counters, int nslices, const double *const *bases,
                        const double *psi, double *y, double *work, double *part, SliceBufs bufs, void *stream);
// wide (WIDE_MB) tiles, s <= WIDE_MAX_SLICES, same queue protocol
void launch_wide_split(int stage, const Tile *tiles, const Seg *segs, const SegS *ssegs, int ntiles,
                       const XcdQueues &q, int32_t *counters, int nslices, const double *const *bases,
                       const double *psi, double *y, double *work, double *part, SliceBufs bufs, void *stream);

}  // namespace dmrg
