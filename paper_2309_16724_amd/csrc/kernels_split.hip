// Split-precision (BF16 slices) kernels for the stripe products of H.psi.
//
// A product C = A B of FP64 operands is computed from fixed-point BF16 slices
// (see SliceJob): C_ij = 2^(e_i + f_j - 16) sum_{t+u <= s-1} sum_k a^t_ik b^u_kj
// with slice t holding digit t at its weight 2^(-8t).  The inner sums run on
// MFMA into FP32 sums per product group d = t + u (exact for the leading
// groups, one rounded sum for the trailing ones, see slice_groups), and every
// split_fold_k terms the sums are folded into FP64 with the line scales.
// FP64 remains for the fold, the scales and the identity segments.
// Lane layouts (lane l, element e/r):
//   v_mfma_f32_16x16x32_bf16: A[l%16][8(l/16)+e], B[8(l/16)+e][l%16], D[4(l/16)+r][l%16];
//   v_mfma_f32_32x32x16_bf16: A[l%32][8(l/32)+e], B[8(l/32)+e][l%32],
//                             D[8(r/4)+4(l/32)+r%4][l%32].
#include <hip/hip_runtime.h>
#include <climits>
#include "plan.hpp"
#include "queue.hpp"

namespace dmrg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ const double *sbase_ptr(int id, const double *const *bases, const double *psi,
                                                   const double *y, const double *work, const double *part) {
  return id == BASE_PSI ? psi : id == BASE_Y ? y : id == BASE_WORK ? work : id == BASE_PART ? part
                                                                                             : bases[id - BASE_OPS];
}

// ------------------------------------------------------------------ slicing
// 2^(-8t), the weight at which slice t stores its digit
static_assert(SLICE_BITS == 8, "digit weights assume 8-bit slices");
__device__ constexpr float digit_weight(int t) {
  return t == 0 ? 1.0f : t == 1 ? 0x1p-8f : t == 2 ? 0x1p-16f : t == 3 ? 0x1p-24f : t == 4 ? 0x1p-32f
                                                                                        : t == 5 ? 0x1p-40f : 0x1p-48f;
}

__global__ void __launch_bounds__(256) slice_kernel(const SliceJob *__restrict__ jobs, int njobs, int ns,
                                                     const double *const *__restrict__ bases,
                                                     const double *__restrict__ psi,
                                                     const double *__restrict__ work, SliceBufs bufs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
    const SliceJob J = jobs[jb];
    const double *src = sbase_ptr(J.src_base, bases, psi, nullptr, work, nullptr) + J.src_off;
    int32_t *exps = bufs.exps[J.dst_buf] + J.exp_off;
    // line lengths fit in 32 bits (checked when the plan is built): the
    // (position, offset) split of an index is a 32-bit division
    const int len = J.npos * J.kbp;
    const int nval = J.npos * J.kb;
    const unsigned kb = (unsigned)J.kb, kbp = (unsigned)J.kbp;
    for (int rho = wave; rho < J.nrho; rho += 4) {
      const double *line = src + (int64_t)rho * J.s_rho;
      // four independent loads in flight per lane
      double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
      auto val = [&](int idx) {
        const unsigned p = (unsigned)idx / kb, kk = (unsigned)idx - p * kb;
        return fabs(line[(int64_t)p * J.s_pos + (int64_t)kk * J.s_k]);
      };
      int idx = lane;
      for (; idx + 192 < nval; idx += 256) {
        const double v0 = val(idx), v1 = val(idx + 64), v2 = val(idx + 128), v3 = val(idx + 192);
        m0 = fmax(m0, v0);
        m1 = fmax(m1, v1);
        m2 = fmax(m2, v2);
        m3 = fmax(m3, v3);
      }
      for (; idx < nval; idx += 64) m0 = fmax(m0, val(idx));
      double m = fmax(fmax(m0, m1), fmax(m2, m3));
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
      int e = 0;
      if (m > 0.0) {
        int ex;
        double mant = frexp(m, &ex);          // m = mant 2^ex, mant in [0.5, 1)
        e = (mant == 0.5) ? ex - 1 : ex;      // smallest e with m <= 2^e
      }
      if (lane == 0) exps[rho] = e;
      // the line starts at a multiple of 8: its slices start at ns times that
      uint16_t *out = bufs.data[J.dst_buf] + (J.dst_off + (int64_t)rho * len) * ns;
      auto slice_out = [&](int idx, double x) {
        double yv = ldexp(x, -e);
        for (int t = 0; t < ns; t++) {
          double a = rint(yv * 256.0);
          yv = yv * 256.0 - a;
          const float af = (float)a * digit_weight(t);   // |a| <= 256 at weight 2^(-8t): exact in BF16
          out[slice_index(idx, t, ns)] = (uint16_t)(__float_as_uint(af) >> 16);
        }
      };
      auto raw = [&](int idx) {
        const unsigned p = (unsigned)idx / kbp, kk = (unsigned)idx - p * kbp;
        return kk < kb ? line[(int64_t)p * J.s_pos + (int64_t)kk * J.s_k] : 0.0;
      };
      int i2 = lane;
      for (; i2 + 192 < len; i2 += 256) {
        const double x0 = raw(i2), x1 = raw(i2 + 64), x2 = raw(i2 + 128), x3 = raw(i2 + 192);
        slice_out(i2, x0);
        slice_out(i2 + 64, x1);
        slice_out(i2 + 128, x2);
        slice_out(i2 + 192, x3);
      }
      for (; i2 < len; i2 += 64) slice_out(i2, raw(i2));
    }
  }
}

// stripe slices, one work group per chunk of TSLICE_CHUNK elements, four
// consecutive elements per thread.  Line lengths, position blocks (kbp), job
// offsets and chunk starts are multiples of 8, so a group of four never
// straddles a line, a position block or a chunk of 8, and the slices of a
// work group's elements are one contiguous range of the slice buffer: they
// are assembled in LDS and written out in whole 16-byte pieces.
static_assert(TSLICE_CHUNK == 4 * 256, "one chunk is 256 threads x 4 elements");
__global__ void __launch_bounds__(256) tslice_kernel(const SliceJob *__restrict__ jobs,
                                                      const TSliceItem *__restrict__ items, int nitems, int ns,
                                                      const double *__restrict__ work, SliceBufs bufs) {
  __shared__ __attribute__((aligned(16))) uint16_t out[TSLICE_CHUNK * 7];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const TSliceItem I = items[it];
    const SliceJob J = jobs[I.job];
    const unsigned kb = (unsigned)J.kb, kbp = (unsigned)J.kbp, len = (unsigned)(J.npos * J.kbp);
    const unsigned tot = len * (unsigned)J.nrho;
    const unsigned n = min((unsigned)TSLICE_CHUNK, tot - (unsigned)I.e0);   // a multiple of 8
    const unsigned el = 4u * threadIdx.x, e = (unsigned)I.e0 + el;
    if (el < n) {
      const unsigned rho = e / len, idx = e - rho * len;
      const unsigned p = idx / kbp, kk = idx - p * kbp;
      const double *line = work + J.src_off + (int64_t)rho * J.s_rho + (int64_t)p * J.s_pos;
      const int ex = bufs.exps[SBUF_T][J.exp_off + rho];
      double yv[4];
      for (int i = 0; i < 4; i++) {
        const unsigned k = kk + i;
        const double x = line[(int64_t)min(k, kb - 1) * J.s_k];    // padding reads a valid entry ...
        yv[i] = ldexp(k < kb ? x : 0.0, ex == INT_MIN ? 0 : -ex);  // ... and slices zero
      }
      for (int t = 0; t < ns; t++) {
        uint64_t packed = 0;
        for (int i = 0; i < 4; i++) {
          const double a = rint(yv[i] * 256.0);
          yv[i] = yv[i] * 256.0 - a;
          const float af = (float)a * digit_weight(t);   // exact in BF16 (see slice_kernel)
          packed |= (uint64_t)(__float_as_uint(af) >> 16) << (16 * i);
        }
        *(uint64_t *)(out + slice_index(el, t, ns)) = packed;
      }
    }
    __syncthreads();
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    v4u *dst = (v4u *)(bufs.data[SBUF_T] + slice_index(J.dst_off + I.e0, 0, ns));
    for (unsigned u = threadIdx.x; u < n * ns / 8; u += blockDim.x) dst[u] = ((const v4u *)out)[u];
    __syncthreads();   // out is reused by the next chunk
  }
}

__global__ void fill_int_kernel(int32_t *__restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_tslices(const SliceJob *jobs, const TSliceItem *items, int nitems, int nslices, const double *work,
                    SliceBufs bufs, void *stream) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(tslice_kernel, dim3(std::min(nitems, 65535)), dim3(256), 0, (hipStream_t)stream, jobs, items,
                     nitems, nslices, work, bufs);
}

void launch_fill_int(int32_t *p, int64_t n, int32_t v, void *stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65535)), dim3(256), 0,
                     (hipStream_t)stream, p, n, v);
}

void launch_slices(const SliceJob *jobs, int njobs, int nslices, const double *const *bases, const double *psi,
                   const double *work, SliceBufs bufs, void *stream) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(slice_kernel, dim3(std::min(njobs, 8192)), dim3(256), 0, (hipStream_t)stream, jobs, njobs,
                     nslices, bases, psi, work, bufs);
}

// ------------------------------------------------------------------ split products
// descriptor arrays read through the constant address space (scalar loads)
typedef const SegS __attribute__((address_space(4))) CSegS;
typedef const Seg __attribute__((address_space(4))) CSeg;
// slice buffers live in device global memory: global (not flat) loads
typedef const void __attribute__((address_space(1))) *gvptr;
typedef void __attribute__((address_space(3))) *lvptr;
typedef const v8bf __attribute__((address_space(3))) *lv8ptr;
// s_waitcnt immediates (gfx9 encoding): vmcnt(0) alone, lgkmcnt(0) alone
constexpr int WAIT_VM0 = 0x0F70, WAIT_LGKM0 = 0xC07F;

// LDS stage of one wavefront: (MB + NB) * NS chunks of 64 lanes x 16 bytes
constexpr int stage_bytes(int ns) { return 5 * ns * 1024; }

// FP32 sum of slice-product group d for s = NS (see slice_groups)
template <int NS>
__device__ constexpr int sgroup(int d) { return d < slice_groups(NS) - 1 ? d : slice_groups(NS) - 1; }
static_assert(SLICE_BITS == 8, "fold weights assume 8-bit slices");

// fold of the group sums of one element: their FP64 sum (group 0 first)
template <int G, typename V>
__device__ __forceinline__ double fold_groups(const V *q, int r) {
  double x = (double)q[0][r];
  for (int g = 1; g < G; g++) x += (double)q[g][r];
  return x;
}

template <int MB, int NS>
__device__ __forceinline__ void item_split(const Tile &T, const Seg *__restrict__ segs,
                                           const SegS *__restrict__ ssegs, const double *const *bases,
                                           const double *psi, double *y, double *work, double *part,
                                           const SliceBufs &bufs, char *stage, int r16, int q4) {
  constexpr int NB = 4 / MB;
  v4d acc[MB][NB];
  for (int a = 0; a < MB; a++)
    for (int b = 0; b < NB; b++) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int mrem = T.m - T.i0, nrem = T.n - T.j0;
  for (int si = 0; si < T.nseg; si++) {
    const Seg S = segs[T.seg0 + si];
    const SegS Q = ssegs[T.seg0 + si];
    if (Q.K == 0) {
      // identity left operator: exact FP64 addition of the FP64 operand
      const double *B = sbase_ptr(S.b_base, bases, psi, y, work, part) + S.b_off;
      for (int bi = 0; bi < MB; bi++)
        for (int bj = 0; bj < NB; bj++) {
          int jj = 16 * bj + r16;
          if (jj >= nrem) continue;
          int n = T.j0 + jj;
          int pn = n / S.b_nb;
          int64_t bo = (int64_t)pn * S.b_pn + (int64_t)(n - pn * S.b_nb) * S.b_n;
          for (int r = 0; r < 4; r++) {
            int i = 16 * bi + 4 * q4 + r;
            if (i < mrem) {
              int k = T.i0 + i;
              int pk = k / S.b_kb;
              acc[bi][bj][r] += S.s * B[(int64_t)pk * S.b_pk + (int64_t)(k - pk * S.b_kb) * S.b_k + bo];
            }
          }
        }
      continue;
    }
    // segment offsets and line lengths are multiples of 8: a segment's slices
    // start at NS times its offset, a line's at NS times its start
    const uint16_t *A = bufs.data[Q.a_buf] + Q.a_off * NS;
    const uint16_t *B = bufs.data[Q.b_buf] + Q.b_off * NS;
    const int32_t *ea = bufs.exps[Q.a_buf] + Q.a_exp;
    const int32_t *eb = bufs.exps[Q.b_buf] + Q.b_exp;
    // lanes past the last row / column read the last one: their outputs are
    // never stored, so every operand load is unconditional.  Addresses are a
    // wave-uniform slice base plus a 32-bit lane offset within the segment's
    // lines (checked when the plan is built).
    uint32_t arow[MB], bcol[NB];   // byte offsets
    for (int bi = 0; bi < MB; bi++)
      arow[bi] = (uint32_t)(T.i0 + min(16 * bi + r16, mrem - 1)) * (uint32_t)Q.a_ld * (2u * NS);
    for (int bj = 0; bj < NB; bj++)
      bcol[bj] = (uint32_t)(T.j0 + min(16 * bj + r16, nrem - 1)) * (uint32_t)Q.b_ld * (2u * NS);
    // scale exponents of this lane's output elements
    int erow[MB][4], fcol[NB];
    for (int bi = 0; bi < MB; bi++)
      for (int r = 0; r < 4; r++) erow[bi][r] = ea[T.i0 + min(16 * bi + 4 * q4 + r, mrem - 1)];
    for (int bj = 0; bj < NB; bj++) fcol[bj] = eb[T.j0 + min(16 * bj + r16, nrem - 1)];
    v4f q[MB][NB][slice_groups(NS)];
    for (int bi = 0; bi < MB; bi++)
      for (int bj = 0; bj < NB; bj++)
        for (int g = 0; g < slice_groups(NS); g++) q[bi][bj][g] = (v4f){0.f, 0.f, 0.f, 0.f};
    // K is a multiple of 8 and the lines are zero-padded to it, so the chunk
    // of 8 at min(k, K - 8) is always inside the operand; a lane whose chunk
    // starts at or past K multiplies a zeroed A operand.  The operands of a
    // step go straight from global memory into this wave's LDS stage (one
    // 1 KiB chunk per operand row block and slice, 16 bytes per lane), so the
    // loads of the next step fly while the MFMAs of this one run without
    // holding a second set of registers.
    auto dma = [&](int k0) {
      const uint32_t kl = (2u * NS) * (uint32_t)min(k0 + 8 * q4, Q.K - 8);
      for (int t = 0; t < NS; t++) {
        const char *at = (const char *)A + 16 * t, *bt = (const char *)B + 16 * t;
        for (int bi = 0; bi < MB; bi++)
          __builtin_amdgcn_global_load_lds((gvptr)(at + (arow[bi] + kl)), (lvptr)(stage + (bi * NS + t) * 1024), 16, 0, 0);
        for (int bj = 0; bj < NB; bj++)
          __builtin_amdgcn_global_load_lds((gvptr)(bt + (bcol[bj] + kl)), (lvptr)(stage + ((MB + bj) * NS + t) * 1024),
                                           16, 0, 0);
      }
    };
    auto rd = [&](v8bf (*as)[NS], v8bf (*bs)[NS]) {
      const int lo = 16 * (r16 + 16 * q4);
      for (int t = 0; t < NS; t++) {
        for (int bi = 0; bi < MB; bi++) as[bi][t] = *(const lv8ptr)(stage + (bi * NS + t) * 1024 + lo);
        for (int bj = 0; bj < NB; bj++) bs[bj][t] = *(const lv8ptr)(stage + ((MB + bj) * NS + t) * 1024 + lo);
      }
    };
    auto mma = [&](int k0, v8bf (*as)[NS], v8bf (*bs)[NS]) {
      if (k0 + 32 > Q.K && k0 + 8 * q4 >= Q.K)   // only the last step of a line has such lanes
        for (int bi = 0; bi < MB; bi++)
          for (int t = 0; t < NS; t++) as[bi][t] = (v8bf){};
#pragma unroll
      for (int d = 0; d < NS; d++)
#pragma unroll
        for (int t = 0; t <= d; t++)
          for (int bi = 0; bi < MB; bi++)
            for (int bj = 0; bj < NB; bj++)
              q[bi][bj][sgroup<NS>(d)] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[bi][t], bs[bj][d - t], q[bi][bj][sgroup<NS>(d)], 0, 0, 0);
    };
    auto fold = [&]() {
      for (int bi = 0; bi < MB; bi++)
        for (int bj = 0; bj < NB; bj++)
          for (int r = 0; r < 4; r++) {
            const double x = fold_groups<slice_groups(NS)>(q[bi][bj], r);
            acc[bi][bj][r] += S.s * ldexp(x, erow[bi][r] + fcol[bj] - 2 * SLICE_BITS);
          }
      for (int bi = 0; bi < MB; bi++)
        for (int bj = 0; bj < NB; bj++)
          for (int g = 0; g < slice_groups(NS); g++) q[bi][bj][g] = (v4f){0.f, 0.f, 0.f, 0.f};
    };
    constexpr int FOLD = split_fold_k(NS);
    static_assert(FOLD % 32 == 0, "the K loop folds after whole 32-wide steps");
    v8bf as[MB][NS], bs[NB][NS];
    dma(0);
    for (int k0 = 0; k0 < Q.K; k0 += 32) {
      __builtin_amdgcn_s_waitcnt(WAIT_VM0);      // this step's chunks are in LDS
      __builtin_amdgcn_sched_barrier(0);
      rd(as, bs);
      __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);    // ... and in registers: the stage is free
      __builtin_amdgcn_sched_barrier(0);
      if (k0 + 32 < Q.K) dma(k0 + 32);
      __builtin_amdgcn_sched_barrier(0);
      mma(k0, as, bs);
      if (k0 + 32 >= Q.K || (k0 + 32) % FOLD == 0) fold();
    }
  }
  double *C = const_cast<double *>(sbase_ptr(T.c_base, bases, psi, y, work, part)) + T.c_off;
  for (int bi = 0; bi < MB; bi++)
    for (int bj = 0; bj < NB; bj++)
      for (int r = 0; r < 4; r++) {
        int i = 16 * bi + 4 * q4 + r, j = 16 * bj + r16;
        if (i < mrem && j < nrem) {
          double *c = T.rowmajor ? C + (int64_t)(T.ci0 + i) * T.ldc + (T.cj0 + j)
                                 : C + (int64_t)(T.ci0 + i) + (int64_t)(T.cj0 + j) * T.ldc;
          *c = T.accumulate ? *c + acc[bi][bj][r] : acc[bi][bj][r];
        }
      }
  // first-stage tiles: exponent of every stripe column they wrote (smallest e
  // with max |value| <= 2^e), combined over tiles with atomicMax
  const SegS Q0 = ssegs[T.seg0];
  if (Q0.t_exp >= 0) {
    int32_t *ex = bufs.exps[SBUF_T] + Q0.t_exp;
    for (int bj = 0; bj < NB; bj++) {
      const int j = 16 * bj + r16;
      double m = 0.0;
      for (int bi = 0; bi < MB; bi++)
        for (int r = 0; r < 4; r++) {
          const int i = 16 * bi + 4 * q4 + r;
          if (i < mrem && j < nrem) m = fmax(m, fabs(acc[bi][bj][r]));
        }
      m = fmax(m, __shfl_xor(m, 16));
      m = fmax(m, __shfl_xor(m, 32));
      if (q4 == 0 && j < nrem && m > 0.0) {
        int e2;
        const double mant = frexp(m, &e2);
        atomicMax(ex + (T.cj0 + j) % Q0.t_nb, mant == 0.5 ? e2 - 1 : e2);
      }
    }
  }
}

// Wavefront tiles: every wavefront takes its next tile from the per-XCD
// queues (one lane takes it, the index is wave-uniform).
template <int NS>
__device__ __forceinline__ void items_split(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,
                                            const SegS *__restrict__ ssegs, const XcdQueues &q,
                                            int32_t *__restrict__ counters,
                                            const double *const *__restrict__ bases, const double *__restrict__ psi,
                                            double *__restrict__ y, double *__restrict__ work,
                                            double *__restrict__ part, const SliceBufs &bufs) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, q4 = lane >> 4;
  __shared__ __attribute__((aligned(1024))) char lds[WAVES * stage_bytes(NS)];
  char *stage = lds + wave * stage_bytes(NS);
  const int x = xcc_id();
  int qi = 0;
  for (;;) {
    int v = -1;
    if (lane == 0) v = queue_next(q, counters, x, qi);
    const int t = __builtin_amdgcn_readfirstlane(v);
    if (t < 0) break;
    const Tile T = tiles[t];
    if (T.mb == 1) item_split<1, NS>(T, segs, ssegs, bases, psi, y, work, part, bufs, stage, r16, q4);
    else if (T.mb == 4) item_split<4, NS>(T, segs, ssegs, bases, psi, y, work, part, bufs, stage, r16, q4);
    else item_split<2, NS>(T, segs, ssegs, bases, psi, y, work, part, bufs, stage, r16, q4);
  }
}

// ------------------------------------------------------------ work-group tiles
// A 64 x 64 output tile computed by the four wavefronts of a work group: wave
// w owns the 32 x 32 quarter (w >> 1, w & 1).  Each 32-wide K step of the
// operands (A: 4 row blocks of 16 rows, B: 4 column blocks of 16 columns, NS
// slices each) goes from global memory straight into one of two LDS stages --
// wave w loads row block w and column block w, 16 bytes per lane and slice,
// in the MFMA operand layout -- and after one barrier every wave reads the two
// row blocks and two column blocks of its quarter.  The loads of the next step
// (across segment boundaries) are issued before this step's MFMAs, so each
// operand byte is fetched once per work group instead of once per wavefront,
// and the stage's waves overlap their loads with the other work group's MFMAs
// (two work groups per CU).
constexpr int mstage_bytes(int ns) { return 8 * ns * 1024; }

template <int NS>
__device__ __forceinline__ void macro_split(const Tile &T, const Seg *__restrict__ segs,
                                            const SegS *__restrict__ ssegs, const double *const *bases,
                                            const double *psi, double *y, double *work, double *part,
                                            const SliceBufs &bufs, char *lds, int wave, int lane) {
  constexpr int MB = 2, NB = 2;
  constexpr int STAGE = mstage_bytes(NS);
  constexpr int FOLD = split_fold_k(NS);
  static_assert(FOLD % 32 == 0, "the K loop folds after whole 32-wide steps");
  const int r16 = lane & 15, q4 = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  const int i0 = T.i0 + 32 * wr, j0 = T.j0 + 32 * wc;     // this wave's quarter
  const int mrem = T.m - i0, nrem = T.n - j0;              // <= 0: quarter outside the output
  // operand line this lane loads (row block `wave` of A, column block `wave` of
  // B); lines past the output read the last one (never stored)
  const uint32_t lrow = (uint32_t)min(T.i0 + 16 * wave + r16, T.m - 1);
  const uint32_t lcol = (uint32_t)min(T.j0 + 16 * wave + r16, T.n - 1);
  v4d acc[MB][NB];
  for (int a = 0; a < MB; a++)
    for (int b = 0; b < NB; b++) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  // identity left operators: exact FP64 additions of the FP64 operand
  for (int si = 0; si < T.nseg; si++) {
    if (ssegs[T.seg0 + si].K != 0) continue;
    const Seg S = segs[T.seg0 + si];
    const double *B = sbase_ptr(S.b_base, bases, psi, y, work, part) + S.b_off;
    for (int bi = 0; bi < MB; bi++)
      for (int bj = 0; bj < NB; bj++) {
        const int jj = 16 * bj + r16;
        if (jj >= nrem) continue;
        const int n = j0 + jj;
        const int pn = n / S.b_nb;
        const int64_t bo = (int64_t)pn * S.b_pn + (int64_t)(n - pn * S.b_nb) * S.b_n;
        for (int r = 0; r < 4; r++) {
          const int i = 16 * bi + 4 * q4 + r;
          if (i < mrem) {
            const int k = i0 + i;
            const int pk = k / S.b_kb;
            acc[bi][bj][r] += S.s * B[(int64_t)pk * S.b_pk + (int64_t)(k - pk * S.b_kb) * S.b_k + bo];
          }
        }
      }
  }
  int si = 0;
  while (si < T.nseg && ssegs[T.seg0 + si].K == 0) si++;
  // every wave has finished reading the LDS stages of its previous tile
  __syncthreads();
  if (si < T.nseg) {
    // scale exponents of this lane's outputs (clamped inside the output)
    auto exps = [&](const SegS &Q, int (*er)[4], int *fc) {
      const int32_t *ea = bufs.exps[Q.a_buf] + Q.a_exp;
      const int32_t *eb = bufs.exps[Q.b_buf] + Q.b_exp;
      for (int bi = 0; bi < MB; bi++)
        for (int r = 0; r < 4; r++) er[bi][r] = ea[min(i0 + 16 * bi + 4 * q4 + r, T.m - 1)];
      for (int bj = 0; bj < NB; bj++) fc[bj] = eb[min(j0 + 16 * bj + r16, T.n - 1)];
    };
    // one K step of segment Q at k0 into LDS stage b (K is a multiple of 8 and
    // lines are zero-padded to it: the chunk of 8 at min(k, K - 8) is inside
    // the operand; lanes whose chunk starts at or past K are zeroed at the MFMA)
    auto issue = [&](const SegS &Q, int k0, int b) {
      const char *A = (const char *)(bufs.data[Q.a_buf] + Q.a_off * NS);   // slices interleaved (see item_split)
      const char *B = (const char *)(bufs.data[Q.b_buf] + Q.b_off * NS);
      const uint32_t kl = (2u * NS) * (uint32_t)min(k0 + 8 * q4, Q.K - 8);
      const uint32_t ao = lrow * (uint32_t)Q.a_ld * (2u * NS) + kl, bo = lcol * (uint32_t)Q.b_ld * (2u * NS) + kl;
      char *st = lds + b * STAGE;
      for (int t = 0; t < NS; t++) {
        __builtin_amdgcn_global_load_lds((gvptr)(A + 16 * t + ao), (lvptr)(st + (wave * NS + t) * 1024), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((gvptr)(B + 16 * t + bo), (lvptr)(st + ((4 + wave) * NS + t) * 1024), 16,
                                         0, 0);
      }
    };
    v4f q[MB][NB][slice_groups(NS)];
    for (int bi = 0; bi < MB; bi++)
      for (int bj = 0; bj < NB; bj++)
        for (int g = 0; g < slice_groups(NS); g++) q[bi][bj][g] = (v4f){0.f, 0.f, 0.f, 0.f};
    SegS Q = ssegs[T.seg0 + si];
    double sc = segs[T.seg0 + si].s;
    int erow[MB][4], fcol[NB];
    exps(Q, erow, fcol);
    issue(Q, 0, 0);
    int k0 = 0, b = 0;
    for (;;) {
      __builtin_amdgcn_s_waitcnt(WAIT_VM0);      // this wave's chunks of the step are in LDS ...
      __syncthreads();                          // ... and every other wave's; the other stage is free
      int nsi = si, nk0 = k0 + 32;
      const bool newseg = nk0 >= Q.K;
      if (newseg) {
        nk0 = 0;
        nsi++;
        while (nsi < T.nseg && ssegs[T.seg0 + nsi].K == 0) nsi++;
      }
      const bool more = nsi < T.nseg;
      SegS NQ = Q;
      double nsc = sc;
      int nerow[MB][4], nfcol[NB];
      if (more && newseg) {
        NQ = ssegs[T.seg0 + nsi];
        nsc = segs[T.seg0 + nsi].s;
      }
      // this step's operands: LDS -> registers, all reads complete (and the
      // next segment's descriptors in) before the next step's loads into the
      // other stage are issued, so no wait below depends on those loads
      v8bf as[MB][NS], bs[NB][NS];
      const char *st = lds + b * STAGE;
      for (int t = 0; t < NS; t++) {
        for (int bi = 0; bi < MB; bi++) as[bi][t] = *(const lv8ptr)(st + ((2 * wr + bi) * NS + t) * 1024 + 16 * lane);
        for (int bj = 0; bj < NB; bj++)
          bs[bj][t] = *(const lv8ptr)(st + ((4 + 2 * wc + bj) * NS + t) * 1024 + 16 * lane);
      }
      __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
      __builtin_amdgcn_sched_barrier(0);
      if (more) {
        issue(NQ, nk0, b ^ 1);
        if (newseg) exps(NQ, nerow, nfcol);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (k0 + 32 > Q.K && k0 + 8 * q4 >= Q.K)   // only the last step of a segment has such lanes
        for (int bi = 0; bi < MB; bi++)
          for (int t = 0; t < NS; t++) as[bi][t] = (v8bf){};
#pragma unroll
      for (int d = 0; d < NS; d++)
#pragma unroll
        for (int t = 0; t <= d; t++)
          for (int bi = 0; bi < MB; bi++)
            for (int bj = 0; bj < NB; bj++)
              q[bi][bj][sgroup<NS>(d)] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[bi][t], bs[bj][d - t], q[bi][bj][sgroup<NS>(d)], 0, 0, 0);
      if (newseg || (k0 + 32) % FOLD == 0) {
        for (int bi = 0; bi < MB; bi++)
          for (int bj = 0; bj < NB; bj++)
            for (int r = 0; r < 4; r++) {
              const double x = fold_groups<slice_groups(NS)>(q[bi][bj], r);
              acc[bi][bj][r] += sc * ldexp(x, erow[bi][r] + fcol[bj] - 2 * SLICE_BITS);
            }
        for (int bi = 0; bi < MB; bi++)
          for (int bj = 0; bj < NB; bj++)
            for (int g = 0; g < slice_groups(NS); g++) q[bi][bj][g] = (v4f){0.f, 0.f, 0.f, 0.f};
      }
      if (!more) break;
      if (newseg) {
        Q = NQ;
        sc = nsc;
        si = nsi;
        for (int bi = 0; bi < MB; bi++)
          for (int r = 0; r < 4; r++) erow[bi][r] = nerow[bi][r];
        for (int bj = 0; bj < NB; bj++) fcol[bj] = nfcol[bj];
      }
      k0 = nk0;
      b ^= 1;
    }
  }
  double *C = const_cast<double *>(sbase_ptr(T.c_base, bases, psi, y, work, part)) + T.c_off;
  const int ci0 = T.ci0 + 32 * wr, cj0 = T.cj0 + 32 * wc;
  for (int bi = 0; bi < MB; bi++)
    for (int bj = 0; bj < NB; bj++)
      for (int r = 0; r < 4; r++) {
        const int i = 16 * bi + 4 * q4 + r, j = 16 * bj + r16;
        if (i < mrem && j < nrem) {
          double *c = T.rowmajor ? C + (int64_t)(ci0 + i) * T.ldc + (cj0 + j)
                                 : C + (int64_t)(ci0 + i) + (int64_t)(cj0 + j) * T.ldc;
          *c = T.accumulate ? *c + acc[bi][bj][r] : acc[bi][bj][r];
        }
      }
  // first-stage tiles: exponent of every stripe column written (see item_split)
  const SegS Q0 = ssegs[T.seg0];
  if (Q0.t_exp >= 0) {
    int32_t *ex = bufs.exps[SBUF_T] + Q0.t_exp;
    for (int bj = 0; bj < NB; bj++) {
      const int j = 16 * bj + r16;
      double m = 0.0;
      for (int bi = 0; bi < MB; bi++)
        for (int r = 0; r < 4; r++) {
          const int i = 16 * bi + 4 * q4 + r;
          if (i < mrem && j < nrem) m = fmax(m, fabs(acc[bi][bj][r]));
        }
      m = fmax(m, __shfl_xor(m, 16));
      m = fmax(m, __shfl_xor(m, 32));
      if (q4 == 0 && j < nrem && m > 0.0) {
        int e2;
        const double mant = frexp(m, &e2);
        atomicMax(ex + (cj0 + j) % Q0.t_nb, mant == 0.5 ? e2 - 1 : e2);
      }
    }
  }
}

template <int NS>
__device__ __forceinline__ void macro_items(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,
                                            const SegS *__restrict__ ssegs, const XcdQueues &q,
                                            int32_t *__restrict__ counters,
                                            const double *const *__restrict__ bases, const double *__restrict__ psi,
                                            double *__restrict__ y, double *__restrict__ work,
                                            double *__restrict__ part, const SliceBufs &bufs) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // all of the LDS holds the two operand stages (two work groups per CU); the
  // tile index taken by thread 0 reaches the other wavefronts through this
  // work group's mailbox in global memory (atomics: coherent at the L2)
  __shared__ __attribute__((aligned(1024))) char lds[2 * mstage_bytes(NS)];
  int32_t *mailbox = counters + NXCD + blockIdx.x;
  const int x = xcc_id();   // this work group's XCD: its own range first
  int qi = 0;               // thread 0's queue state
  for (;;) {
    if (threadIdx.x == 0) atomicExch(mailbox, queue_next(q, counters, x, qi));
    // every wave reads the mailbox before the barrier inside macro_split, the
    // earliest point where thread 0 can write it again
    __syncthreads();
    int v = 0;
    if (lane == 0) v = atomicAdd(mailbox, 0);
    const int t = __builtin_amdgcn_readfirstlane(v);
    if (t < 0) break;   // every queue is empty: the whole work group leaves
    const Tile T = tiles[t];
    macro_split<NS>(T, segs, ssegs, bases, psi, y, work, part, bufs, lds, wave, lane);
  }
}

#define MACRO_KERNELS(NS)                                                                                   \
  __global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))                 \
  stage1_msplit##NS##_kernel(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,                  \
                             const SegS *__restrict__ ssegs, XcdQueues q, int32_t *__restrict__ counters,   \
                             const double *const *__restrict__ bases, const double *__restrict__ psi,       \
                             double *__restrict__ y, double *__restrict__ work, double *__restrict__ part,   \
                             SliceBufs bufs) {                                                              \
    macro_items<NS>(tiles, segs, ssegs, q, counters, bases, psi, y, work, part, bufs);                      \
  }                                                                                                         \
  __global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))                 \
  stage2_msplit##NS##_kernel(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,                  \
                             const SegS *__restrict__ ssegs, XcdQueues q, int32_t *__restrict__ counters,   \
                             const double *const *__restrict__ bases, const double *__restrict__ psi,       \
                             double *__restrict__ y, double *__restrict__ work, double *__restrict__ part,   \
                             SliceBufs bufs) {                                                              \
    macro_items<NS>(tiles, segs, ssegs, q, counters, bases, psi, y, work, part, bufs);                      \
  }

MACRO_KERNELS(3)
MACRO_KERNELS(4)
MACRO_KERNELS(5)
MACRO_KERNELS(6)
MACRO_KERNELS(7)

// ------------------------------------------------------------ wide work-group tiles
// A 128 x 128 output tile (WIDE_MB) computed by the eight wavefronts of a
// work group, two per SIMD: wave w owns rows 32 (w >> 1) .. + 32 and columns
// 64 (w & 1) .. + 64 as two blocks of v_mfma_f32_32x32x16_bf16.  The MFMA
// takes the B lines (output columns) as its first operand and the A lines
// (output rows) as its second, so lane l holds output row l % 32 of a block
// and its columns wcol(r) = 8 (r / 4) + 4 (l / 32) + r % 4: the column-major
// stores of 32 lanes are contiguous 256-byte runs.  Each 32-wide K step of
// the operands (A: 4 row blocks of 32 lines, B: 4 column blocks, two K halves
// of 16, NS slices; 1 KiB per block, half and slice) goes from global memory
// through registers into one of two LDS stages -- wave w loads row block
// w % 4 and column block w % 4 of K half w / 4 -- while the step before runs
// on the other stage.  The stages are two separate LDS objects, so the
// compiler knows that the stores into one never alias the reads of the other.
constexpr int wstage_bytes(int ns) { return 16 * ns * 1024; }
__device__ __forceinline__ int wcol(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

template <int NS>
__device__ __forceinline__ void wide_split(const Tile &T, const Seg *__restrict__ segs,
                                           const SegS *__restrict__ ssegs, const double *const *bases,
                                           const double *psi, double *y, double *work, double *part,
                                           const SliceBufs &bufs, char *lds0, char *lds1, int wave, int lane) {
  constexpr int FOLD = split_fold_k(NS);
  static_assert(FOLD % 32 == 0, "the K loop folds after whole 32-wide steps");
  typedef float v16f __attribute__((ext_vector_type(16)));
  // the tile and segment descriptors do not change during the launch: read
  // through the constant address space they are scalar loads (scalar cache,
  // no vector memory wait on the K loop's path)
  const CSegS *cs = (const CSegS *)ssegs;
  const CSeg *cg = (const CSeg *)segs;
  // the lane index passes through an empty asm per tile: the per-lane column
  // offsets derived from it are recomputed per tile instead of being hoisted
  // out of the tile loop into registers that the K loop needs
  asm volatile("" : "+v"(lane));
  const int c32 = lane & 31, h = lane >> 5;
  const int wr = wave >> 1, wc = wave & 1;
  const int i0 = T.i0 + 32 * wr, j0 = T.j0 + 64 * wc;    // this wave's part
  const int mrem = T.m - i0, nrem = T.n - j0;             // <= 0: part outside the output
  // operand lines this lane loads: row block / column block wave % 4, K half
  // wave / 4 (see issue)
  const int lb = wave & 3, lkh = wave >> 2;
  double acc[2][16];
  for (int bj = 0; bj < 2; bj++)
    for (int r = 0; r < 16; r++) acc[bj][r] = 0.0;
  // identity left operators: exact FP64 additions of the FP64 operand
  for (int si = 0; si < T.nseg; si++) {
    if (cs[T.seg0 + si].K != 0) continue;
    CSeg &S = cg[T.seg0 + si];
    const double *B = sbase_ptr(S.b_base, bases, psi, y, work, part) + S.b_off;
    if (c32 >= mrem) continue;
    const int k = i0 + c32;
    const int pk = k / S.b_kb;
    const int64_t ko = (int64_t)pk * S.b_pk + (int64_t)(k - pk * S.b_kb) * S.b_k;
    for (int bj = 0; bj < 2; bj++)
      for (int r = 0; r < 16; r++) {
        const int j = 32 * bj + wcol(r, h);
        if (j < nrem) {
          const int n = j0 + j;
          const int pn = n / S.b_nb;
          acc[bj][r] += S.s * B[ko + (int64_t)pn * S.b_pn + (int64_t)(n - pn * S.b_nb) * S.b_n];
        }
      }
  }
  int si = 0;
  while (si < T.nseg && cs[T.seg0 + si].K == 0) si++;
  // every wave has finished reading the LDS stages of its previous tile
  __syncthreads();
  if (si < T.nseg) {
    // one operand's NS chunks of a K step of segment qi at k0 (operand 0: the A
    // lines of row block wave % 4, 1: the B lines of column block wave % 4; K
    // half wave / 4) into registers.  K is a multiple of 8 and lines are
    // zero-padded to it: the chunk of 8 at min(k, K - 8) is inside the operand;
    // lanes whose chunk starts at or past K are zeroed at the MFMA.  Plain
    // vector loads: under load they complete about 2.5 times sooner than
    // loads straight into LDS.
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    auto load = [&](int qi, int k0, int op, v4u *pre) {
      CSegS &Q = cs[T.seg0 + qi];
      const int buf = op ? Q.b_buf : Q.a_buf;
      const char *X = (const char *)(bufs.data[buf] + (op ? Q.b_off : Q.a_off) * NS);   // see item_split
      // the lane index is recomputed here (volatile: not kept in a register
      // across the K loop); lines past the output read the last one (never stored)
      int ln;
      asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
      const uint32_t line = (uint32_t)(op ? min(T.j0 + 32 * lb + (ln & 31), T.n - 1)
                                          : min(T.i0 + 32 * lb + (ln & 31), T.m - 1));
      const uint32_t kl = (2u * NS) * (uint32_t)min(k0 + 16 * lkh + 8 * (ln >> 5), Q.K - 8);
      const uint32_t xo = line * (uint32_t)(op ? Q.b_ld : Q.a_ld) * (2u * NS) + kl;
      for (int t = 0; t < NS; t++) pre[t] = *(const v4u *)(X + xo + 16 * t);
    };
    // ... and from registers into LDS stage st, in the MFMA operand layout
    auto store = [&](int op, const v4u *pre, char *st) {
      int ln;
      asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
      for (int t = 0; t < NS; t++)
        *(v4u *)(st + (8 * NS * op + (2 * lb + lkh) * NS + t) * 1024 + 16 * ln) = pre[t];
    };
    v16f q[2][slice_groups(NS)];
    for (int bj = 0; bj < 2; bj++)
      for (int g = 0; g < slice_groups(NS); g++) q[bj][g] = (v16f){};
    // one K half kh of this step's products from stage st: the row block's A
    // slices, then per column block its B slices one at a time (slice u
    // meets A slices t <= NS - 1 - u), the next one read while the MFMAs of
    // the current one run; so only five A and two B operands are in registers
    auto compute = [&](const char *st, int k0, int K, int kh) {
      v8bf a[NS];
      for (int t = 0; t < NS; t++) a[t] = *(const lv8ptr)(st + ((2 * wr + kh) * NS + t) * 1024 + 16 * lane);
      if (k0 + 32 > K && k0 + 16 * kh + 8 * h >= K)   // only a segment's last step has such lanes
        for (int t = 0; t < NS; t++) a[t] = (v8bf){};
      for (int bj = 0; bj < 2; bj++) {
        const char *bs = st + (8 * NS + (2 * (2 * wc + bj) + kh) * NS) * 1024 + 16 * lane;
        v8bf b = *(const lv8ptr)bs;
#pragma unroll
        for (int u = 0; u < NS; u++) {
          const v8bf bn = u + 1 < NS ? *(const lv8ptr)(bs + (u + 1) * 1024) : b;
#pragma unroll
          for (int t = 0; t + u < NS; t++)
            q[bj][sgroup<NS>(t + u)] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a[t], q[bj][sgroup<NS>(t + u)], 0, 0, 0);
          b = bn;
        }
      }
    };
    // segment descriptors are read where needed (wave-uniform, scalar loads)
    // rather than copied, so that they never sit in scratch memory
    // fold into FP64 with the scale exponents of this lane's row and its 32
    // columns, read here (the exponent arrays hold WIDE_EDGE spare entries, so
    // the lines past the output read in bounds; their outputs are never
    // stored).  Exponents are in [-1100, 1100] or the all-zero sentinel, which
    // only meets zero sums: int16 keeps every sum of two in range.
    auto fold = [&]() {
      CSegS &Q = cs[T.seg0 + si];
      const double sc = cg[T.seg0 + si].s;
      const int32_t *ea = bufs.exps[Q.a_buf] + Q.a_exp + (i0 + c32);
      const int32_t *eb = bufs.exps[Q.b_buf] + Q.b_exp + (j0 + 4 * h);
      const int er = (int16_t)ea[0];
      for (int bj = 0; bj < 2; bj++)
        for (int r = 0; r < 16; r++) {
          const int f = (int16_t)eb[32 * bj + 8 * (r >> 2) + (r & 3)];
          const double x = fold_groups<slice_groups(NS)>(q[bj], r);
          acc[bj][r] += sc * ldexp(x, er + f - 2 * SLICE_BITS);
        }
      for (int bj = 0; bj < 2; bj++)
        for (int g = 0; g < slice_groups(NS); g++) q[bj][g] = (v16f){};
    };
    {
      v4u pre[NS];
      load(si, 0, 0, pre);
      store(0, pre, lds0);
      load(si, 0, 1, pre);
      store(1, pre, lds0);
    }
    int k0 = 0;
    // one step on stage cur; the next one (across segment boundaries) goes
    // through registers into nxt, its loads in flight during the whole step.
    // Returns false after the tile's last step.
    auto step = [&](const char *cur, char *nxt) -> bool {
      __syncthreads();   // every wave's chunks of this step are in cur; nxt is free
      const int K = cs[T.seg0 + si].K;
      int nsi = si, nk0 = k0 + 32;
      const bool newseg = nk0 >= K;
      if (newseg) {
        nk0 = 0;
        nsi++;
        while (nsi < T.nseg && cs[T.seg0 + nsi].K == 0) nsi++;
      }
      const bool more = nsi < T.nseg;
      v4u pa[NS], pb[NS];
      if (more) {
        load(nsi, nk0, 0, pa);
        load(nsi, nk0, 1, pb);
      }
      compute(cur, k0, K, 0);
      compute(cur, k0, K, 1);
      __builtin_amdgcn_sched_barrier(0);
      if (more) {
        store(0, pa, nxt);
        store(1, pb, nxt);
      }
      if (newseg || (k0 + 32) % FOLD == 0) fold();
      si = nsi;
      k0 = nk0;
      return more;
    };
    while (step(lds0, lds1) && step(lds1, lds0)) {
    }
  }
  double *C = const_cast<double *>(sbase_ptr(T.c_base, bases, psi, y, work, part)) + T.c_off;
  const int ci0 = T.ci0 + 32 * wr, cj0 = T.cj0 + 64 * wc;
  for (int bj = 0; bj < 2; bj++)
    for (int r = 0; r < 16; r++) {
      const int i = c32, j = 32 * bj + wcol(r, h);
      if (i < mrem && j < nrem) {
        double *c = T.rowmajor ? C + (int64_t)(ci0 + i) * T.ldc + (cj0 + j)
                               : C + (int64_t)(ci0 + i) + (int64_t)(cj0 + j) * T.ldc;
        *c = T.accumulate ? *c + acc[bj][r] : acc[bj][r];
      }
    }
  // first-stage tiles: exponent of every stripe column written (see
  // item_split), the maximum of the elements' exponents over the rows
  CSegS &Q0 = cs[T.seg0];
  if (Q0.t_exp >= 0) {
    int32_t *ex = bufs.exps[SBUF_T] + Q0.t_exp;
    for (int bj = 0; bj < 2; bj++)
      for (int r = 0; r < 16; r++) {
        const int j = 32 * bj + wcol(r, h);
        const double m = fabs(acc[bj][r]);
        int e = INT_MIN;
        if (c32 < mrem && j < nrem && m > 0.0) {
          int e2;
          const double mant = frexp(m, &e2);
          e = mant == 0.5 ? e2 - 1 : e2;
        }
        for (int off = 16; off > 0; off >>= 1) e = max(e, __shfl_xor(e, off));
        if (c32 == 0 && j < nrem && e != INT_MIN) atomicMax(ex + (cj0 + j) % Q0.t_nb, e);
      }
  }
}

template <int NS>
__device__ __forceinline__ void wide_items(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,
                                           const SegS *__restrict__ ssegs, const XcdQueues &q,
                                           int32_t *__restrict__ counters,
                                           const double *const *__restrict__ bases, const double *__restrict__ psi,
                                           double *__restrict__ y, double *__restrict__ work,
                                           double *__restrict__ part, const SliceBufs &bufs) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the two operand stages fill the LDS (one work group of eight wavefronts
  // per CU); the tile index reaches the wavefronts through the work group's
  // mailbox as in macro_items
  __shared__ __attribute__((aligned(1024))) char lds0[wstage_bytes(NS)];
  __shared__ __attribute__((aligned(1024))) char lds1[wstage_bytes(NS)];
  int32_t *mailbox = counters + NXCD + blockIdx.x;
  const int x = xcc_id();
  int qi = 0;
  for (;;) {
    if (threadIdx.x == 0) atomicExch(mailbox, queue_next(q, counters, x, qi));
    __syncthreads();
    int v = 0;
    if (lane == 0) v = atomicAdd(mailbox, 0);
    const int t = __builtin_amdgcn_readfirstlane(v);
    if (t < 0) break;
    const Tile T = tiles[t];
    wide_split<NS>(T, segs, ssegs, bases, psi, y, work, part, bufs, lds0, lds1, wave, lane);
  }
}

#define WIDE_KERNELS(NS)                                                                                    \
  __global__ void __launch_bounds__(64 * WIDE_WAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))           \
  stage1_wsplit##NS##_kernel(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,                  \
                             const SegS *__restrict__ ssegs, XcdQueues q, int32_t *__restrict__ counters,   \
                             const double *const *__restrict__ bases, const double *__restrict__ psi,       \
                             double *__restrict__ y, double *__restrict__ work, double *__restrict__ part,   \
                             SliceBufs bufs) {                                                              \
    wide_items<NS>(tiles, segs, ssegs, q, counters, bases, psi, y, work, part, bufs);                       \
  }                                                                                                         \
  __global__ void __launch_bounds__(64 * WIDE_WAVES) __attribute__((amdgpu_waves_per_eu(2, 2)))           \
  stage2_wsplit##NS##_kernel(const Tile *__restrict__ tiles, const Seg *__restrict__ segs,                  \
                             const SegS *__restrict__ ssegs, XcdQueues q, int32_t *__restrict__ counters,   \
                             const double *const *__restrict__ bases, const double *__restrict__ psi,       \
                             double *__restrict__ y, double *__restrict__ work, double *__restrict__ part,   \
                             SliceBufs bufs) {                                                              \
    wide_items<NS>(tiles, segs, ssegs, q, counters, bases, psi, y, work, part, bufs);                       \
  }

WIDE_KERNELS(3)
WIDE_KERNELS(4)
WIDE_KERNELS(5)

#define SPLIT_KERNELS(NS)                                                                                   \
  __global__ void __launch_bounds__(64 * WAVES) stage1_split##NS##_kernel(                                  \
      const Tile *__restrict__ tiles, const Seg *__restrict__ segs, const SegS *__restrict__ ssegs,         \
      XcdQueues q, int32_t *__restrict__ counters, const double *const *__restrict__ bases,                 \
      const double *__restrict__ psi, double *__restrict__ y, double *__restrict__ work,                    \
      double *__restrict__ part, SliceBufs bufs) {                                                          \
    items_split<NS>(tiles, segs, ssegs, q, counters, bases, psi, y, work, part, bufs);                      \
  }                                                                                                         \
  __global__ void __launch_bounds__(64 * WAVES) stage2_split##NS##_kernel(                                  \
      const Tile *__restrict__ tiles, const Seg *__restrict__ segs, const SegS *__restrict__ ssegs,         \
      XcdQueues q, int32_t *__restrict__ counters, const double *const *__restrict__ bases,                 \
      const double *__restrict__ psi, double *__restrict__ y, double *__restrict__ work,                    \
      double *__restrict__ part, SliceBufs bufs) {                                                          \
    items_split<NS>(tiles, segs, ssegs, q, counters, bases, psi, y, work, part, bufs);                      \
  }

SPLIT_KERNELS(3)
SPLIT_KERNELS(4)
SPLIT_KERNELS(5)
SPLIT_KERNELS(6)
SPLIT_KERNELS(7)

void launch_macro_split(int stage, const Tile *tiles, const Seg *segs, const SegS *ssegs, int ntiles,
                        const XcdQueues &q, int32_t *counters, int nslices, const double *const *bases,
                        const double *psi, double *y, double *work, double *part, SliceBufs bufs, void *stream) {
  if (ntiles <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, counters, (int64_t)NXCD, 0);
  // two work groups resident per CU (80 KiB of LDS each at s = 5); every work
  // group takes tiles until all queues are empty
  const int grid = std::max(8, std::min((ntiles + 7) / 8 * 8, MACRO_GRID));
#define MLAUNCH(NS)                                                                                         \
  if (nslices == NS) {                                                                                      \
    if (stage == 1)                                                                                         \
      hipLaunchKernelGGL(stage1_msplit##NS##_kernel, dim3(grid), dim3(64 * WAVES), 0, s, tiles, segs, ssegs,  \
                         q, counters, bases, psi, y, work, part, bufs);                                     \
    else                                                                                                    \
      hipLaunchKernelGGL(stage2_msplit##NS##_kernel, dim3(grid), dim3(64 * WAVES), 0, s, tiles, segs, ssegs,  \
                         q, counters, bases, psi, y, work, part, bufs);                                     \
    return;                                                                                                 \
  }
  MLAUNCH(3)
  MLAUNCH(4)
  MLAUNCH(5)
  MLAUNCH(6)
  MLAUNCH(7)
#undef MLAUNCH
}

void launch_wide_split(int stage, const Tile *tiles, const Seg *segs, const SegS *ssegs, int ntiles,
                       const XcdQueues &q, int32_t *counters, int nslices, const double *const *bases,
                       const double *psi, double *y, double *work, double *part, SliceBufs bufs, void *stream) {
  if (ntiles <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, counters, (int64_t)NXCD, 0);
  // one work group per CU (the two stages take all 160 KiB of LDS at s = 5)
  const int grid = std::max(8, std::min((ntiles + 7) / 8 * 8, WIDE_GRID));
#define WLAUNCH(NS)                                                                                         \
  if (nslices == NS) {                                                                                      \
    if (stage == 1)                                                                                         \
      hipLaunchKernelGGL(stage1_wsplit##NS##_kernel, dim3(grid), dim3(64 * WIDE_WAVES), 0, s, tiles, segs,  \
                         ssegs, q, counters, bases, psi, y, work, part, bufs);                              \
    else                                                                                                    \
      hipLaunchKernelGGL(stage2_wsplit##NS##_kernel, dim3(grid), dim3(64 * WIDE_WAVES), 0, s, tiles, segs,  \
                         ssegs, q, counters, bases, psi, y, work, part, bufs);                              \
    return;                                                                                                 \
  }
  WLAUNCH(3)
  WLAUNCH(4)
  WLAUNCH(5)
#undef WLAUNCH
}

void launch_tiles_split(int stage, const Tile *tiles, const Seg *segs, const SegS *ssegs, int ntiles,
                        const XcdQueues &q, int32_t *counters, int nslices, const double *const *bases,
                        const double *psi, double *y, double *work, double *part, SliceBufs bufs, void *stream) {
  if (ntiles <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, counters, (int64_t)NXCD, 0);
  int grid = std::min((ntiles + WAVES - 1) / WAVES, 256 * 16);
  grid = (grid + 7) / 8 * 8;
#define LAUNCH(NS)                                                                                          \
  if (nslices == NS) {                                                                                      \
    if (stage == 1)                                                                                         \
      hipLaunchKernelGGL(stage1_split##NS##_kernel, dim3(grid), dim3(64 * WAVES), 0, s, tiles, segs, ssegs,   \
                         q, counters, bases, psi, y, work, part, bufs);                                     \
    else                                                                                                    \
      hipLaunchKernelGGL(stage2_split##NS##_kernel, dim3(grid), dim3(64 * WAVES), 0, s, tiles, segs, ssegs,   \
                         q, counters, bases, psi, y, work, part, bufs);                                     \
    return;                                                                                                 \
  }
  LAUNCH(3)
  LAUNCH(4)
  LAUNCH(5)
  LAUNCH(6)
  LAUNCH(7)
#undef LAUNCH
}

}  // namespace dmrg
