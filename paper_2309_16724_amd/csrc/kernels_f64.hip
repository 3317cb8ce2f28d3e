// FP64 MFMA kernels for the grouped stripe products of H.psi.
//
// Every H.psi is two launches of one work-item routine.  The first stage
// computes, for each wavefunction block X and run of right-block operator
// positions, T = X [op(D_1) ... op(D_c)] (positions concatenated along N).
// The second stage accumulates Y_F += sum v [A_1 ... A_c] [T_1; ...; T_c] for
// every output block F.  Output tiles are owned by work items; a tile whose
// segment list is long is split into parts (split K) that write partial
// tiles, summed afterwards in a fixed order, so no atomics are used and the
// result is bitwise reproducible.  A wavefront handles one work item: a
// (16 mb) x (64/mb) tile as mb x (4/mb) v_mfma_f64_16x16x4 products with
// operands loaded into registers one K step ahead.
// Lane layout of v_mfma_f64_16x16x4f64 (lane l, accumulator element r):
// A[l%16][l/16], B[l/16][l%16], D[l/16 + 4r][l%16].
#include <hip/hip_runtime.h>
#include <algorithm>
#include "plan.hpp"
#include "queue.hpp"

namespace dmrg {

typedef double v4d __attribute__((ext_vector_type(4)));


// Operand pointers come from a table of generic pointers; every one of them
// addresses device global memory, and saying so lets the compiler emit global
// (not flat) loads, whose counters allow waiting for the oldest loads only --
// otherwise each wait drains every load in flight and the prefetch is lost.
typedef const double __attribute__((address_space(1))) *gcptr;
typedef double __attribute__((address_space(1))) *gptr;
__device__ __forceinline__ double gld(const double *p) { return *(gcptr)p; }


__device__ __forceinline__ const double *base_ptr(int id, const double *const *bases, const double *psi,
                                                  const double *y, const double *work, const double *part) {
  return id == BASE_PSI ? psi : id == BASE_Y ? y : id == BASE_WORK ? work : id == BASE_PART ? part
                                                                                             : bases[id - BASE_OPS];
}

// One work item: tile of MB x NB MFMA blocks (MB * NB == 4).
template <int MB>
__device__ __forceinline__ void item_f64(const Tile &T, const Seg *__restrict__ segs, const double *const *bases,
                                         const double *psi, double *y, double *work, double *part, int r16,
                                         int q4) {
  constexpr int NB = 4 / MB;
  v4d acc[MB][NB];
  for (int a = 0; a < MB; a++)
    for (int b = 0; b < NB; b++) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int mrem = T.m - T.i0, nrem = T.n - T.j0;
  for (int si = 0; si < T.nseg; si++) {
    const Seg S = segs[T.seg0 + si];
    const double *B = base_ptr(S.b_base, bases, psi, y, work, part) + S.b_off;
    int64_t boff[NB];
    bool bok[NB];
    for (int bj = 0; bj < NB; bj++) {
      int n = T.j0 + 16 * bj + r16;
      bok[bj] = (16 * bj + r16) < nrem;
      int pn = bok[bj] ? n / S.b_nb : 0;
      boff[bj] = bok[bj] ? (int64_t)pn * S.b_pn + (int64_t)(n - pn * S.b_nb) * S.b_n : 0;
    }
    if (S.a_base < 0) {
      // identity left operator: tile += s * B restricted to the tile (K == rows)
      for (int bi = 0; bi < MB; bi++)
        for (int bj = 0; bj < NB; bj++)
          for (int r = 0; r < 4; r++) {
            int i = 16 * bi + q4 + 4 * r;
            if (i < mrem && bok[bj]) {
              int k = T.i0 + i;
              int pk = k / S.b_kb;
              acc[bi][bj][r] += S.s * gld(B + (int64_t)pk * S.b_pk + (int64_t)(k - pk * S.b_kb) * S.b_k + boff[bj]);
            }
          }
      continue;
    }
    const double *A = base_ptr(S.a_base, bases, psi, y, work, part) + S.a_off;
    int64_t aoff[MB];
    bool aok[MB];
    for (int bi = 0; bi < MB; bi++) {
      aok[bi] = (16 * bi + r16) < mrem;
      aoff[bi] = aok[bi] ? (int64_t)(T.i0 + 16 * bi + r16) * S.a_i : 0;
    }
    const double s = S.s;
    // Two operand buffers of one K step each, used alternately: while the
    // matrix core works on one, the loads of the next-but-one step fill the
    // other.  The loop is unrolled by two so the buffers are never copied (a
    // copy would wait for the loads just issued), and no load depends on a
    // condition: lanes outside the tile read an element inside the operand
    // (their outputs are never stored), and lanes past the end of K read
    // element K-1 and scale it by zero instead of s (operands are finite).
    const unsigned akb = (unsigned)S.a_kb, bkb = (unsigned)S.b_kb;
    auto step = [&](int k0, const double *an, const double *bn) {
      const double sk = k0 + q4 < S.K ? s : 0.0;
      double ac[MB];
      for (int bi = 0; bi < MB; bi++) ac[bi] = sk * an[bi];
      for (int bi = 0; bi < MB; bi++)
        for (int bj = 0; bj < NB; bj++)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[bi], bn[bj], acc[bi][bj], 0, 0, 0);
    };
    // scheduling barriers keep each buffer's refill in program order, so the
    // older buffer's loads are always the ones waited for; one exit: a second
    // half past K contributes zero (its scale is zero)
    auto kloop = [&](auto &&fetch) {
      double a0[MB], b0[NB], a1[MB], b1[NB];
      fetch(0, a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      fetch(4, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      for (int k0 = 0; k0 < S.K; k0 += 8) {
        step(k0, a0, b0);
        fetch(k0 + 8, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        step(k0 + 4, a1, b1);
        fetch(k0 + 12, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    if (akb >= 4 && bkb >= 4) {
      // A lane's K index k0 + q4 moves by 4 per step and crosses at most one
      // position boundary, so its (position, offset) pairs are carried along
      // with adds and selects; lanes at or past K read element K - 1, whose
      // offsets are wave-uniform.
      const unsigned kl = (unsigned)S.K - 1, pla = kl / akb, plb = kl / bkb;
      const int64_t al = (int64_t)pla * S.a_p + (int64_t)(kl - pla * akb) * S.a_k;
      const int64_t bl = (int64_t)plb * S.b_pk + (int64_t)(kl - plb * bkb) * S.b_k;
      const int64_t ad = 4 * S.a_k, aw = S.a_p - (int64_t)akb * S.a_k;
      const int64_t bd = 4 * S.b_k, bw = S.b_pk - (int64_t)bkb * S.b_k;
      unsigned ka = q4, kb = q4;
      int64_t ao = (int64_t)q4 * S.a_k, bo = (int64_t)q4 * S.b_k;
      kloop([&](int k0, double *an, double *bn) {
        int64_t ua = ao, ub = bo;
        if (k0 + 4 > S.K && k0 + q4 >= S.K) {
          ua = al;
          ub = bl;
        }
        for (int bi = 0; bi < MB; bi++) an[bi] = gld(A + ua + aoff[bi]);
        for (int bj = 0; bj < NB; bj++) bn[bj] = gld(B + ub + boff[bj]);
        ka += 4;
        ao += ad;
        if (ka >= akb) {
          ka -= akb;
          ao += aw;
        }
        kb += 4;
        bo += bd;
        if (kb >= bkb) {
          kb -= bkb;
          bo += bw;
        }
      });
    } else {
      kloop([&](int k0, double *an, double *bn) {
        const int k = min(k0 + q4, S.K - 1);
        const unsigned pa = (unsigned)k / akb, ka = (unsigned)k - pa * akb;
        const unsigned pb = (unsigned)k / bkb, kb = (unsigned)k - pb * bkb;
        const int64_t ak = (int64_t)pa * S.a_p + (int64_t)ka * S.a_k;
        const int64_t bk = (int64_t)pb * S.b_pk + (int64_t)kb * S.b_k;
        for (int bi = 0; bi < MB; bi++) an[bi] = gld(A + ak + aoff[bi]);
        for (int bj = 0; bj < NB; bj++) bn[bj] = gld(B + bk + boff[bj]);
      });
    }
  }
  double *C = const_cast<double *>(base_ptr(T.c_base, bases, psi, y, work, part)) + T.c_off;
  for (int bi = 0; bi < MB; bi++)
    for (int bj = 0; bj < NB; bj++)
      for (int r = 0; r < 4; r++) {
        int i = 16 * bi + q4 + 4 * r, j = 16 * bj + r16;
        if (i < mrem && j < nrem) {
          gptr c = (gptr)(T.rowmajor ? C + (int64_t)(T.ci0 + i) * T.ldc + (T.cj0 + j)
                                     : C + (int64_t)(T.ci0 + i) + (int64_t)(T.cj0 + j) * T.ldc);
          *c = T.accumulate ? *c + acc[bi][bj][r] : acc[bi][bj][r];
        }
      }
}

// One launch per stage: every wavefront takes tiles from the per-XCD queues
// of the stage's cost-sorted list and runs the work item of the tile's shape.
// Three wavefronts per SIMD (at most 168 registers, no spills): more loads in
// flight per SIMD than the two that the register use of an unbounded build
// allows; four spill.
template <int STAGE>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(3, 3))) stage_f64_kernel(
    const Tile *__restrict__ tiles, const Seg *__restrict__ segs, XcdQueues q, int32_t *__restrict__ counters,
    const double *const *__restrict__ bases, const double *__restrict__ psi, double *__restrict__ y,
    double *__restrict__ work, double *__restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int x = xcc_id();
  int qi = 0;
  for (;;) {
    // the tile index is the same for the whole wavefront: saying so makes the
    // descriptors scalar loads and the K loops uniform (no exec masking)
    int v = -1;
    if (lane == 0) v = queue_next(q, counters, x, qi);
    const int t = __builtin_amdgcn_readfirstlane(v);
    if (t < 0) break;
    const Tile T = tiles[t];
    if (T.mb == 1) item_f64<1>(T, segs, bases, psi, y, work, part, r16, q4);
    else if (T.mb == 4) item_f64<4>(T, segs, bases, psi, y, work, part, r16, q4);
    else item_f64<2>(T, segs, bases, psi, y, work, part, r16, q4);
  }
}

// Y tile += sum of its partial tiles, in part order
// one output tile per blockIdx.x (grid-stride), its elements shared by the
// REDUCE_SPLIT blocks along y: the 128 x 128 tiles of wide plans have 16384
// elements, which one block of 256 threads would take alone
constexpr int REDUCE_SPLIT = 16;
__global__ void reduce_kernel(const Reduce *__restrict__ red, int nred, const double *__restrict__ part,
                              double *__restrict__ y) {
  for (int r = blockIdx.x; r < nred; r += gridDim.x) {
    const Reduce R = red[r];
    int mt = min(R.tm, R.m - R.i0);
    int nt = min(R.tn, R.n - R.j0);
    const int64_t ps = (int64_t)R.tm * R.tn;
    for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < mt * nt; e += gridDim.y * blockDim.x) {
      int i = e % mt, j = e / mt;
      double v = 0.0;
      for (int p = 0; p < R.nparts; p++) v += part[R.part_off + (int64_t)p * ps + i + (int64_t)j * R.tm];
      y[R.y_off + (int64_t)(R.i0 + i) + (int64_t)(R.j0 + j) * R.ldc] += v;
    }
  }
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

// dressed right-block operators (once per plan)
__global__ void dress_kernel(const DressItem *__restrict__ items, int nitems,
                             const int64_t *__restrict__ src_off, const double *__restrict__ alpha,
                             const double *const *__restrict__ bases, double *__restrict__ dst) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const DressItem D = items[it];
    const double *src = bases[D.src_base - BASE_OPS];
    for (int64_t e = threadIdx.x; e < D.n; e += blockDim.x) {
      double acc = 0.0;
      for (int t = D.t0; t < D.t1; t++) acc += alpha[t] * src[src_off[t] + e];
      dst[D.dst_off + e] = acc;
    }
  }
}

void launch_dress(const DressItem *items, int nitems, const int64_t *src_off, const double *alpha,
                  const double *const *bases, double *dst, void *stream) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(dress_kernel, dim3(std::min(nitems, 8192)), dim3(256), 0, (hipStream_t)stream, items,
                     nitems, src_off, alpha, bases, dst);
}

void launch_zero(double *y, int64_t n, void *stream) {
  if (n <= 0) return;
  int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, y, n);
}

void launch_tiles_f64(int stage, const Tile *tiles, const Seg *segs, int ntiles, const XcdQueues &q,
                      int32_t *counters, const double *const *bases, const double *psi, double *y, double *work,
                      double *part, void *stream) {
  if (ntiles <= 0) return;
  hipStream_t s = (hipStream_t)stream;
  launch_fill_int(counters, NXCD, 0, stream);
  int grid = std::min((ntiles + WAVES - 1) / WAVES, 256 * 16);
  grid = (grid + 7) / 8 * 8;
  if (stage == 1)
    hipLaunchKernelGGL(stage_f64_kernel<1>, dim3(grid), dim3(64 * WAVES), 0, s, tiles, segs, q, counters, bases,
                       psi, y, work, part);
  else
    hipLaunchKernelGGL(stage_f64_kernel<2>, dim3(grid), dim3(64 * WAVES), 0, s, tiles, segs, q, counters, bases,
                       psi, y, work, part);
}

void launch_reduce(const Reduce *red, int nred, const double *part, double *y, void *stream) {
  if (nred <= 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3(std::min(nred, 8192), REDUCE_SPLIT), dim3(256), 0, (hipStream_t)stream, red,
                     nred, part, y);
}

void launch_diag(const DiagBlock *blocks, const DiagTerm *terms, int nblocks, const double *const *bases,
                 double *diag, void *stream) {
  if (nblocks <= 0) return;
  int grid = std::min(nblocks, 4096);
  hipLaunchKernelGGL(diag_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, blocks, terms, nblocks,
                     bases, diag);
}

// dst block (c, r) = src block (r, c) for every position of every job
__global__ void __launch_bounds__(256) transpose_kernel(const TransJob *__restrict__ jobs, int njobs,
                                                        const double *__restrict__ src, double *__restrict__ dst) {
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    const TransJob J = jobs[j];
    const int64_t bs = (int64_t)J.rows * J.cols, tot = bs * J.npos;
    for (int64_t e = threadIdx.x; e < tot; e += 256) {
      const int64_t p = e / bs, rem = e - p * bs;
      const int64_t c = rem / J.rows, r = rem - c * J.rows;
      dst[J.off + p * bs + c + r * J.cols] = src[J.off + e];
    }
  }
}

void launch_transpose(const TransJob *jobs, int njobs, const double *src, double *dst, void *stream) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(transpose_kernel, dim3(std::min(njobs, 65535)), dim3(256), 0, (hipStream_t)stream, jobs, njobs,
                     src, dst);
}

}  // namespace dmrg
