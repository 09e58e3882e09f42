/*
 * dsrg_testing.h -- test entry points of libdsrg (not needed by applications).
 *
 * dsrg_test_gett runs the library's strided contraction kernel once on host arrays:
 *   C[m][n] = alpha * sum_k A[m][k] B[k][n] + (beta ? C[m][n] : 0)
 * where m, n, k are multi-indices with nm, nn, nk (<= 6) components of extents md, nd,
 * kd (row-major composition), and each operand addresses element (m, k), (k, n), (m, n)
 * through its own per-component strides (am, ak), (bk, bn), (cm, cn) in elements.
 * na, nb, nc are the host array lengths (elements), which must cover every addressed
 * element.  The caller owns every buffer; C is read (beta != 0) and overwritten.
 * precision selects the kernel: DSRG_PRECISION_FP64, DSRG_PRECISION_FP32 (FP32 products)
 * or DSRG_PRECISION_BF16X3 (split-BF16 products), the last two with FP64 accumulation
 * between k chunks (see dsrg.h).
 * Returns DSRG_OK or a DSRG_E_* code (message in dsrg_last_error).
 */
#ifndef DSRG_TESTING_H
#define DSRG_TESTING_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif
int dsrg_test_gett(int nm, const int* md, const long long* am, const long long* cm,
                   int nn, const int* nd, const long long* bn, const long long* cn,
                   int nk, const int* kd, const long long* ak, const long long* bk,
                   const double* A, long long na, const double* B, long long nb,
                   double* C, long long nc, double alpha, int beta, int precision);
/* Loss (mean squared error of the standardised targets) and its gradient with respect to
   every parameter (grad: DSRG_MLP_WEIGHTS_BYTES / 4 - 64 floats, in the blob's parameter
   order) of the pair-energy network at the given weights, computed by the training
   kernels (forward, backward) on the GPU.  Host arrays. */
int dsrg_test_mlp_grad(const void* weights, const float* X, const double* y, int64_t n, double* loss,
                       float* grad);
#ifdef __cplusplus
}
#endif
#endif
