// Davidson solver: device vector kernels (kernels_vec.hip) and the host loop.
#pragma once
#include <cstdint>

namespace dmrg {
void vec_dots(const double *V, int64_t ldv, int m, const double *x, int64_t n, double *part, double *out,
              void *stream);
int64_t vec_dots_part_len(int64_t n, int m);
void vec_combo(const double *V, int64_t ldv, int m, const double *c, double sign, double beta, double *y,
               int64_t n, void *stream);
void vec_resid(const double *hu, const double *u, const double *diag, double theta, double floor_, double *r,
               double *t, int64_t n, void *stream);
void vec_scale(double *x, double s, int64_t n, void *stream);
// cyclic Jacobi eigensolver of a symmetric m x m matrix (row-major); returns
// eigenvalues ascending in w and the matching eigenvectors as columns of Z
void jacobi_eigh(int m, const double *A, double *w, double *Z);
}  // namespace dmrg
