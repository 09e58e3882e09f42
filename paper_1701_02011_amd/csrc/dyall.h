// Active-to-virtual doubles under Dyall's zeroth-order Hamiltonian (App. B, Eq. t2_aavv).
// Internal interface between the entry point (dsrg.hip) and the kernels (dyall.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace dsrg_dyall {

// Largest active space solved: a block of the alpha-beta system holds nA^2 unknowns and is
// factorised in LDS as an nA^2 x (nA^2 + 1) FP64 array (53 KB at nA = 9).
constexpr int kMaxActive = 9;

// The active coupling of Eq. t2_aavv as matrices over the unknowns of one virtual pair:
// Kaa, Kbb [np][np] over unique pairs u < v (row-major pair order, np = nA(nA-1)/2) and
// Kab [nA^2][nA^2] over ordered (u alpha, v beta); rows are outputs, columns inputs.
// Jaaaa[x][u][y][v] = (xu|yv); g1 [2][nA][nA] with g1[s][y][z] = <a+_y a_z>.
void launch_operator(int nA, const double* Jaaaa, const double* g1, double* Kaa, double* Kbb,
                     double* Kab, hipStream_t st);

// Solves (Delta + K) t = v for every virtual pair and spin block by Gaussian elimination
// with partial pivoting, one workgroup per block.  eps [N] (core, active, virtual),
// Jvava[e][u][f][v] = (eu|fv); t [3][nV][nV][nA][nA] (blocks aa, ab, bb, t[e][f][u][v],
// antisymmetric in the same-spin blocks); dmin [3 nV^2] the smallest |diagonal| of each
// block (+inf where no block is solved); singular[0] is set to 1 when a pivot falls below
// 1e-13 of the block's largest element (that block's amplitudes are then NaN).
void launch_solve(int nC, int nA, int nV, const double* eps, const double* Jvava, const double* Kaa,
                  const double* Kbb, const double* Kab, double* t, double* dmin, int* singular,
                  hipStream_t st);

// out[0] = min over n values of dmin (one workgroup).
void launch_min(const double* dmin, long long n, double* out, hipStream_t st);

}  // namespace dsrg_dyall
