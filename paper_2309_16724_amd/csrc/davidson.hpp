// Davidson solver: segmented device vector kernels (kernels_vec.hip) and
// the host loop (davidson.cpp).
#pragma once
#include <cstdint>

namespace dmrg {

constexpr int64_t VCHUNK = 1024;   // vector elements per chunk (enough chunks to fill the chip)

struct VChunk {
  int64_t i0, i1;   // element range, inside one segment
  int32_t seg, pad;
};

// device chunk table of a concatenated vector and a partial-sum buffer
struct VecCtx {
  const VChunk *chunks;
  int nchunks;
  const int32_t *seg_chunk0;   // [nseg + 1] first chunk of every segment
  int nseg;
  double *part;                // >= nchunks * (max m) doubles
};

void vec_dots(const VecCtx &X, const double *V, int64_t ldv, int m, const double *x, double *out, void *stream);
void vec_combo(const VecCtx &X, const double *V, int64_t ldv, int m, const double *coef, int ldc, double sign,
               double beta, double *y, void *stream);
// floors: per-segment absolute denominator floors
void vec_resid(const VecCtx &X, const double *hu, const double *u, const double *diag, const double *theta,
               const double *floors, double *r, double *t, void *stream);
void vec_scale(const VecCtx &X, const double *s, double *x, void *stream);
void vec_fill(const VecCtx &X, double value, double *x, void *stream);
void vec_select(const VecCtx &X, const double *flag, const double *src, double *dst, void *stream);
// cyclic Jacobi eigensolver of a symmetric m x m matrix (row-major); returns
// eigenvalues ascending in w and the matching eigenvectors as columns of Z,
// and the number of sweeps that changed the matrix (JACOBI_MAX_SWEEPS when
// the limit stopped it)
constexpr int JACOBI_MAX_SWEEPS = 100;
int jacobi_eigh(int m, const double *A, double *w, double *Z);
}  // namespace dmrg
