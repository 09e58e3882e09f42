// One-step reference relaxation after E(3): the CAS eigenproblem of the summed
// third-order transformed Hamiltonian (Sec. II.B Eq. E_relaxed; App. A).  Internal
// interface between the pipeline (dsrg.hip) and the CAS kernels (cas.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <vector>

namespace dsrg_cas {

struct Err : std::runtime_error {
  int code;
  Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Device inputs after the pipeline: the orbital energies and factorised integrals, the
// active densities, the energies [E(2), E(3)_a, E(3)_b] and the active blocks R of
// [H~(1), A(1)] + [H~(2)_{1,2}, A(1)] + [H~(1), A(2)] (use R of the contraction table:
// R1 [2][nA][nA] then R2 [3][nA]^4, blocks aa, ab, bb).
struct In {
  int nC = 0, nA = 0, nV = 0, M = 0;
  const double* eps = nullptr;       // [N]
  const double* B = nullptr;         // [M][N][N]
  const double* g1 = nullptr;        // [2][nA][nA]
  const double* g2 = nullptr;        // [3][nA]^4
  const double* energies = nullptr;  // [3]
  const double* R = nullptr;         // [2 nA^2 + 3 nA^4]
  int n_alpha = 0, n_beta = 0;
  const double* ci_guess = nullptr;  // host [strings_alpha][strings_beta] or null
};

struct Out {
  double lambda = 0;     // lowest eigenvalue of H_CAS (E(2) + E(3) + relaxation, no E0)
  double cconst = 0;     // scalar of H_CAS
  double residual = 0;   // eigenvector residual norm at exit
  int n_det = 0, iterations = 0, converged = 0;
  std::vector<double> ci, h1, h2, c;   // filled when requested
};

// Runs on st and synchronises it before returning.  want_ci / want_blocks copy the
// eigenvector and the active blocks (h1, h2, c) to the host.
void relax(const In& in, hipStream_t st, bool want_ci, bool want_blocks, Out& out);

}  // namespace dsrg_cas
