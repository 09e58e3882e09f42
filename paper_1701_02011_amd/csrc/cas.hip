// One-step reference relaxation (Sec. II.B Eqs. energy_relaxed, E_relaxed; App. A Eqs.
// Hbar_mb, Hbar_DNO, c0_cas): from the active blocks of the summed third-order transformed
// Hamiltonian, the CAS operator in true-vacuum order and the lowest eigenvalue of its
// determinant matrix.
//
//   Hbar^u_v   = f_u delta_uv + R1 / 2                 (H(0), and the 1/2 of Eqs. Hbar_2nd/3rd)
//   Hbar^uv_xy = <uv||xy> + R2 / 2                      (H(1) two-body, same)
// with R the active blocks of [H~(1), A(1)] + [H~(2)_{1,2}, A(1)] + [H~(1), A(2)] from the
// contraction table; f(1) has no active-active element and [H(0), A] none at all.  Then,
// in spin blocks (aa, ab, bb; the mixed terms of the spin-orbital sums collected on ab):
//   const  = E(2) + E(3) - sum_s sum_uv Hbar_s^u_v g_s^u_v
//            - sum_{s=a,b} sum (Hbar_ss g2_ss / 4 - Hbar_ss^uv_xy g_s^u_x g_s^v_y)
//            - sum (Hbar_ab g2_ab - 2 Hbar_ab^uv_xy g_a^u_x g_b^v_y)
//   c_a^u_v = Hbar_a^u_v - sum_xy Hbar_aa^ux_vy g_a^x_y - sum_xy Hbar_ab^ux_vy g_b^x_y
//   c_b^u_v = Hbar_b^u_v - sum_xy Hbar_bb^ux_vy g_b^x_y - sum_xy Hbar_ab^xu_yv g_a^x_y
// and H_CAS = const + sum c a+a + 1/4 sum Hbar^uv_xy a+_u a+_v a_y a_x over determinants
// |I_alpha J_beta> (alpha creators, then beta creators, ascending, on the vacuum; strings
// in lexicographic order, alpha index slowest).  The matrix is formed element by element
// with the Slater-Condon rules and its lowest eigenpair found by Davidson iterations with
// the diagonal preconditioner; the Rayleigh-Ritz step diagonalises the subspace matrix by
// cyclic Jacobi rotations in one workgroup.
#include "../../include/dsrg.h"
#include "cas.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <string>
#include <vector>

namespace dsrg_cas {

#define CCHECK(x)                                                                            \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) {                                                                  \
      (void)hipGetLastError();                                                               \
      throw Err(e_ == hipErrorOutOfMemory ? DSRG_E_OOM : DSRG_E_HIP,                         \
                std::string(#x) + ": " + hipGetErrorString(e_));                            \
    }                                                                                        \
  } while (0)

constexpr int kMaxSub = 32;        // Davidson subspace (restart size)
constexpr int kMaxIter = 400;
constexpr double kResTol = 1e-9;   // residual norm (E_h) for convergence

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Active blocks of Hbar^[3]_{1,2}: one thread per element of h1 [2][nA][nA] then h2 [3][nA]^4.
__global__ void hbar_active_kernel(int nA, int nC, int N, int M, const double* __restrict__ eps,
                                   const double* __restrict__ B, const double* __restrict__ R,
                                   double* __restrict__ h1, double* __restrict__ h2) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n2 = (long long)nA * nA, n1 = 2 * n2, n4 = n2 * n2;
  if (t < n1) {
    const int u = (int)((t / nA) % nA), v = (int)(t % nA);
    h1[t] = (u == v ? eps[nC + u] : 0.0) + 0.5 * R[t];
    return;
  }
  t -= n1;
  if (t >= 3 * n4) return;
  const int b = (int)(t / n4);
  const long long e = t % n4;
  const int y = (int)(e % nA), x = (int)((e / nA) % nA), v = (int)((e / n2) % nA), u = (int)(e / (n2 * nA));
  const long long NN = (long long)N * N;
  const long long ux = (long long)(nC + u) * N + nC + x, vy = (long long)(nC + v) * N + nC + y;
  const long long uy = (long long)(nC + u) * N + nC + y, vx = (long long)(nC + v) * N + nC + x;
  double j1 = 0.0, j2 = 0.0;
  for (int q = 0; q < M; ++q) {
    const double* Bq = B + (long long)q * NN;
    j1 += Bq[ux] * Bq[vy];
    j2 += Bq[uy] * Bq[vx];
  }
  // <uv||xy> = (ux|vy) - (uy|vx) for equal spins, (ux|vy) for the ab block
  h2[t] = (b == 1 ? j1 : j1 - j2) + 0.5 * R[n1 + t];
}

// Block-wide sum over 256 threads (fixed order: deterministic).
__device__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// c [2][nA][nA] and the scalar of H_CAS; one block of 256 threads.
__global__ __launch_bounds__(256) void cas_operator_kernel(int nA, const double* __restrict__ h1,
                                                           const double* __restrict__ h2,
                                                           const double* __restrict__ g1,
                                                           const double* __restrict__ g2,
                                                           const double* __restrict__ energies,
                                                           double* __restrict__ c, double* __restrict__ cconst) {
  __shared__ double sh[256];
  const int n2 = nA * nA;
  const long long n4 = (long long)n2 * n2;
  const double* hab = h2 + n4;
  for (int t = threadIdx.x; t < 2 * n2; t += blockDim.x) {
    const int s = t / n2, u = (t / nA) % nA, v = t % nA;
    const double* gs = g1 + s * n2;
    const double* go = g1 + (1 - s) * n2;
    const double* hs = h2 + (s == 0 ? 0 : 2 * n4);
    double acc = h1[t];
    for (int x = 0; x < nA; ++x)
      for (int y = 0; y < nA; ++y) {
        acc -= hs[(((long long)u * nA + x) * nA + v) * nA + y] * gs[x * nA + y];
        const double m = s == 0 ? hab[(((long long)u * nA + x) * nA + v) * nA + y]
                                : hab[(((long long)x * nA + u) * nA + y) * nA + v];
        acc -= m * go[x * nA + y];
      }
    c[t] = acc;
  }
  double acc = 0.0;
  for (long long t = threadIdx.x; t < 2 * n2 + 3 * n4; t += blockDim.x) {
    if (t < 2 * n2) {
      acc -= h1[t] * g1[t];
      continue;
    }
    const long long e = t - 2 * n2;
    const int b = (int)(e / n4);
    const long long r = e % n4;
    const int y = (int)(r % nA), x = (int)((r / nA) % nA), v = (int)((r / n2) % nA), u = (int)(r / ((long long)n2 * nA));
    const double* gl = g1 + (b == 2 ? n2 : 0);   // spin of (u, x)
    const double* gr = g1 + (b == 0 ? 0 : n2);   // spin of (v, y)
    const double h = h2[e], pp = gl[u * nA + x] * gr[v * nA + y];
    if (b == 1) acc -= h * g2[e] - 2.0 * h * pp;
    else acc -= 0.25 * h * g2[e] - h * pp;
  }
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) cconst[0] = energies[0] + energies[1] + energies[2] + tot;
}

// spin orbital k = spin * nA + orbital
__device__ __forceinline__ double c_so(int nA, const double* c, int p, int q) {
  const int sp = p / nA, sq = q / nA;
  if (sp != sq) return 0.0;
  return c[(sp * nA + p % nA) * nA + q % nA];
}

// antisymmetrised element Hbar^{pq}_{rs} of spin orbitals from the spin blocks
__device__ __forceinline__ double w_so(int nA, const double* h2, int p, int q, int r, int s) {
  const long long n4 = (long long)nA * nA * nA * nA;
  const int sp = p / nA, sq = q / nA, sr = r / nA, ss = s / nA;
  const int op = p % nA, oq = q % nA, orr = r % nA, os = s % nA;
  auto at = [&](int b, int a0, int a1, int a2, int a3) {
    return h2[b * n4 + (((long long)a0 * nA + a1) * nA + a2) * nA + a3];
  };
  if (sp == sq) {
    if (sr != sp || ss != sp) return 0.0;
    return at(sp == 0 ? 0 : 2, op, oq, orr, os);
  }
  if (sp == 0) {   // p alpha, q beta
    if (sr == 0 && ss == 1) return at(1, op, oq, orr, os);
    if (sr == 1 && ss == 0) return -at(1, op, oq, os, orr);
    return 0.0;
  }
  if (sr == 1 && ss == 0) return at(1, oq, op, os, orr);   // p beta, q alpha
  if (sr == 0 && ss == 1) return -at(1, oq, op, orr, os);
  return 0.0;
}

// sign of a+_k or a_k on determinant D: (-1)^(occupied spin orbitals below k)
__device__ __forceinline__ int below_sign(uint32_t D, int k) {
  return (__popc(D & ((1u << k) - 1u)) & 1) ? -1 : 1;
}

// Determinant matrix of H_CAS, element (i, j) = <D_i| H_CAS |D_j> by the Slater-Condon rules.
__global__ void cas_matrix_kernel(int nA, int nsa, int nsb, const uint32_t* __restrict__ sa,
                                  const uint32_t* __restrict__ sb, const double* __restrict__ c,
                                  const double* __restrict__ h2, const double* __restrict__ cconst,
                                  double* __restrict__ mat) {
  const long long d = (long long)nsa * nsb;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d * d) return;
  const long long i = t / d, j = t % d;
  const uint32_t Di = sa[i / nsb] | (sb[i % nsb] << nA);
  const uint32_t Dj = sa[j / nsb] | (sb[j % nsb] << nA);
  const uint32_t diff = Di ^ Dj;
  const int nd = __popc(diff);
  const int n2 = 2 * nA;
  double val = 0.0;
  if (nd == 0) {
    val = cconst[0];
    for (int k = 0; k < n2; ++k) {
      if (!((Dj >> k) & 1u)) continue;
      val += c_so(nA, c, k, k);
      for (int l = 0; l < n2; ++l)
        if (l != k && ((Dj >> l) & 1u)) val += 0.5 * w_so(nA, h2, k, l, k, l);
    }
  } else if (nd == 2) {
    const uint32_t out = diff & Dj, in = diff & Di;
    const int q = __ffs(out) - 1, p = __ffs(in) - 1;
    // a+_p a_q |D_j>
    uint32_t D = Dj;
    int sg = below_sign(D, q);
    D ^= 1u << q;
    sg *= below_sign(D, p);
    double acc = c_so(nA, c, p, q);
    for (int r = 0; r < n2; ++r)
      if ((Dj >> r) & 1u && r != q) acc += w_so(nA, h2, p, r, q, r);
    val = sg * acc;
  } else if (nd == 4) {
    uint32_t out = diff & Dj, in = diff & Di;
    const int r = __ffs(out) - 1;
    out &= out - 1;
    const int s = __ffs(out) - 1;
    const int p = __ffs(in) - 1;
    in &= in - 1;
    const int q = __ffs(in) - 1;
    // a+_p a+_q a_s a_r |D_j>, r < s, p < q
    uint32_t D = Dj;
    int sg = below_sign(D, r);
    D ^= 1u << r;
    sg *= below_sign(D, s);
    D ^= 1u << s;
    sg *= below_sign(D, q);
    D ^= 1u << q;
    sg *= below_sign(D, p);
    val = sg * w_so(nA, h2, p, q, r, s);
  }
  mat[i * d + j] = val;
}

__global__ void diag_kernel(long long d, const double* __restrict__ mat, double* __restrict__ dg) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d) dg[i] = mat[i * d + i];
}

// w = M v: one 64-lane wave per row, lanes over columns, fixed-order wave reduction.
__global__ __launch_bounds__(256) void gemv_kernel(long long d, const double* __restrict__ mat,
                                                   const double* __restrict__ v, double* __restrict__ w) {
  const long long row = (long long)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= d) return;
  const double* m = mat + row * d;
  double acc = 0.0;
  for (long long j = lane; j < d; j += 64) acc += m[j] * v[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) w[row] = acc;
}

// S[i][col] = S[col][i] = V[i] . W[col] for i <= col; one block per i.
__global__ __launch_bounds__(256) void dots_kernel(long long d, int col, int ld, const double* __restrict__ V,
                                                   const double* __restrict__ W, double* __restrict__ S) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  const double* a = V + (long long)i * d;
  const double* b = W + (long long)col * d;
  double acc = 0.0;
  for (long long j = threadIdx.x; j < d; j += 256) acc += a[j] * b[j];
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) {
    S[i * ld + col] = tot;
    S[col * ld + i] = tot;
  }
}

// Lowest eigenpair of the symmetric k x k matrix S (leading dimension ld) by cyclic Jacobi
// rotations; one block of 64 threads, thread l owning row/column l.  out[0] = eigenvalue,
// y = eigenvector.
__global__ __launch_bounds__(64) void jacobi_lowest_kernel(int k, int ld, const double* __restrict__ S,
                                                           double* __restrict__ y, double* __restrict__ out) {
  __shared__ double A[kMaxSub][kMaxSub + 1];
  __shared__ double Q[kMaxSub][kMaxSub + 1];
  __shared__ double cs[2];
  __shared__ int done;
  const int l = threadIdx.x;
  for (int e = l; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    A[i][j] = 0.5 * (S[i * ld + j] + S[j * ld + i]);
    Q[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (l == 0) {
      double off = 0.0, dia = 0.0;
      for (int i = 0; i < k; ++i) {
        dia += A[i][i] * A[i][i];
        for (int j = i + 1; j < k; ++j) off += A[i][j] * A[i][j];
      }
      done = off <= 1e-32 * (dia + 1e-300);
    }
    __syncthreads();
    if (done) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        if (l == 0) {
          const double apq = A[p][q];
          if (std::fabs(apq) <= 1e-300) {
            cs[0] = 1.0;
            cs[1] = 0.0;
          } else {
            const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
            const double cc = 1.0 / std::sqrt(t * t + 1.0);
            cs[0] = cc;
            cs[1] = t * cc;
          }
        }
        __syncthreads();
        const double cc = cs[0], ss = cs[1];
        if (ss != 0.0) {
          if (l < k) {   // rows p, q: A <- J^T A
            const double ap = A[p][l], aq = A[q][l];
            A[p][l] = cc * ap - ss * aq;
            A[q][l] = ss * ap + cc * aq;
          }
          __syncthreads();
          if (l < k) {   // columns p, q: A <- A J, Q <- Q J
            const double ap = A[l][p], aq = A[l][q];
            A[l][p] = cc * ap - ss * aq;
            A[l][q] = ss * ap + cc * aq;
            const double qp = Q[l][p], qq = Q[l][q];
            Q[l][p] = cc * qp - ss * qq;
            Q[l][q] = ss * qp + cc * qq;
          }
        }
        __syncthreads();
      }
  }
  if (l == 0) {
    int m = 0;
    for (int i = 1; i < k; ++i)
      if (A[i][i] < A[m][m]) m = i;
    done = m;
    out[0] = A[m][m];
  }
  __syncthreads();
  if (l < k) y[l] = Q[l][done];
}

// x = V y, wx = W y, r = wx - theta x
__global__ void ritz_kernel(long long d, int k, const double* __restrict__ V, const double* __restrict__ W,
                            const double* __restrict__ y, const double* __restrict__ theta, double* __restrict__ x,
                            double* __restrict__ wx, double* __restrict__ r) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < k; ++i) {
    a += y[i] * V[(long long)i * d + j];
    b += y[i] * W[(long long)i * d + j];
  }
  x[j] = a;
  wx[j] = b;
  r[j] = b - theta[0] * a;
}

// out[1] = |r|^2 (one block of 256 threads)
__global__ __launch_bounds__(256) void sumsq_kernel(long long d, const double* __restrict__ r, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long j = threadIdx.x; j < d; j += 256) acc += r[j] * r[j];
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) out[1] = tot;
}

// Davidson correction t = r / (theta - diag), the denominator kept away from zero.
__global__ void precond_kernel(long long d, const double* __restrict__ r, const double* __restrict__ dg,
                               const double* __restrict__ theta, double* __restrict__ t) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double den = theta[0] - dg[j];
  if (std::fabs(den) < 1e-6) den = den < 0 ? -1e-6 : 1e-6;
  t[j] = r[j] / den;
}

// Orthogonalise t against V[0..k) (classical Gram-Schmidt, twice), then write t / |t| to
// dst and |t| to out[2]; one block of 256 threads.
__global__ __launch_bounds__(256) void orth_append_kernel(long long d, int k, const double* __restrict__ V,
                                                          double* __restrict__ t, double* __restrict__ dst,
                                                          double* __restrict__ out) {
  __shared__ double sh[256];
  __shared__ double coef[kMaxSub];
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = 0; i < k; ++i) {
      const double* v = V + (long long)i * d;
      double acc = 0.0;
      for (long long j = threadIdx.x; j < d; j += 256) acc += v[j] * t[j];
      const double tot = block_sum256(acc, sh);
      if (threadIdx.x == 0) coef[i] = tot;
    }
    __syncthreads();
    for (long long j = threadIdx.x; j < d; j += 256) {
      double a = t[j];
      for (int i = 0; i < k; ++i) a -= coef[i] * V[(long long)i * d + j];
      t[j] = a;
    }
    __syncthreads();
  }
  double acc = 0.0;
  for (long long j = threadIdx.x; j < d; j += 256) acc += t[j] * t[j];
  const double nrm = std::sqrt(block_sum256(acc, sh));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (long long j = threadIdx.x; j < d; j += 256) dst[j] = t[j] * inv;
  if (threadIdx.x == 0) out[2] = nrm;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
struct Buf {
  hipStream_t st;
  std::vector<void*> p;
  explicit Buf(hipStream_t s) : st(s) {}
  ~Buf() {
    (void)hipStreamSynchronize(st);
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  T* alloc(size_t n) {
    void* q = nullptr;
    CCHECK(hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
    p.push_back(q);
    return static_cast<T*>(q);
  }
};

static std::vector<uint32_t> strings(int n, int k) {
  std::vector<uint32_t> out;
  if (k < 0 || k > n) return out;
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  while (true) {
    uint32_t m = 0;
    for (int i : idx) m |= 1u << i;
    out.push_back(m);
    int i = k - 1;
    while (i >= 0 && idx[i] == n - k + i) --i;
    if (i < 0) break;
    ++idx[i];
    for (int j = i + 1; j < k; ++j) idx[j] = idx[j - 1] + 1;
  }
  return out;
}

static unsigned blocks_of(long long n, int per) { return (unsigned)((n + per - 1) / per); }

void relax(const In& in, hipStream_t st, bool want_ci, bool want_blocks, Out& out) {
  const int nA = in.nA;
  const int N = in.nC + in.nA + in.nV;
  Buf buf(st);
  if (nA == 0) {
    double e[3];
    CCHECK(hipMemcpyAsync(e, in.energies, sizeof(e), hipMemcpyDeviceToHost, st));
    CCHECK(hipStreamSynchronize(st));
    out.lambda = out.cconst = e[0] + e[1] + e[2];
    out.n_det = 1;
    out.converged = 1;
    if (want_ci) out.ci.assign(1, 1.0);
    return;
  }
  const long long n2 = (long long)nA * nA, n4 = n2 * n2;
  double* h1 = buf.alloc<double>(2 * n2);
  double* h2 = buf.alloc<double>(3 * n4);
  double* c = buf.alloc<double>(2 * n2);
  double* scal = buf.alloc<double>(8);   // [0] theta, [1] |r|^2, [2] |t|, [3] const
  hipLaunchKernelGGL(hbar_active_kernel, dim3(blocks_of(2 * n2 + 3 * n4, 256)), dim3(256), 0, st, nA, in.nC, N,
                     in.M, in.eps, in.B, in.R, h1, h2);
  hipLaunchKernelGGL(cas_operator_kernel, dim3(1), dim3(256), 0, st, nA, h1, h2, in.g1, in.g2, in.energies, c,
                     scal + 3);
  CCHECK(hipGetLastError());
  const std::vector<uint32_t> sa = strings(nA, in.n_alpha), sb = strings(nA, in.n_beta);
  const long long d = (long long)sa.size() * sb.size();
  if (d < 1) throw Err(DSRG_E_ARG, "empty determinant space");
  out.n_det = (int)d;
  uint32_t* dsa = buf.alloc<uint32_t>(sa.size());
  uint32_t* dsb = buf.alloc<uint32_t>(sb.size());
  CCHECK(hipMemcpyAsync(dsa, sa.data(), sa.size() * 4, hipMemcpyHostToDevice, st));
  CCHECK(hipMemcpyAsync(dsb, sb.data(), sb.size() * 4, hipMemcpyHostToDevice, st));
  double* mat = buf.alloc<double>((size_t)(d * d));
  hipLaunchKernelGGL(cas_matrix_kernel, dim3(blocks_of(d * d, 256)), dim3(256), 0, st, nA, (int)sa.size(),
                     (int)sb.size(), dsa, dsb, c, h2, scal + 3, mat);
  double* dg = buf.alloc<double>((size_t)d);
  hipLaunchKernelGGL(diag_kernel, dim3(blocks_of(d, 256)), dim3(256), 0, st, d, mat, dg);
  CCHECK(hipGetLastError());
  if (want_blocks) {
    out.h1.resize(2 * n2);
    out.h2.resize(3 * n4);
    out.c.resize(2 * n2);
    CCHECK(hipMemcpyAsync(out.h1.data(), h1, 2 * n2 * 8, hipMemcpyDeviceToHost, st));
    CCHECK(hipMemcpyAsync(out.h2.data(), h2, 3 * n4 * 8, hipMemcpyDeviceToHost, st));
    CCHECK(hipMemcpyAsync(out.c.data(), c, 2 * n2 * 8, hipMemcpyDeviceToHost, st));
  }
  // start vectors: the caller's guess, then unit vectors on the lowest diagonal elements
  std::vector<double> dgh((size_t)d);
  double hc = 0;
  CCHECK(hipMemcpyAsync(dgh.data(), dg, d * 8, hipMemcpyDeviceToHost, st));
  CCHECK(hipMemcpyAsync(&hc, scal + 3, 8, hipMemcpyDeviceToHost, st));
  CCHECK(hipStreamSynchronize(st));
  out.cconst = hc;
  std::vector<long long> order((size_t)d);
  std::iota(order.begin(), order.end(), 0LL);
  std::stable_sort(order.begin(), order.end(), [&](long long a, long long b) { return dgh[a] < dgh[b]; });
  std::vector<std::vector<double>> guesses;
  if (in.ci_guess) guesses.emplace_back(in.ci_guess, in.ci_guess + d);
  for (long long k = 0; k < std::min<long long>(d, 4); ++k) {
    std::vector<double> g((size_t)d, 0.0);
    g[order[k]] = 1.0;
    guesses.push_back(g);
  }
  const int kmax = (int)std::min<long long>(kMaxSub, d);
  double* V = buf.alloc<double>((size_t)(kmax * d));
  double* W = buf.alloc<double>((size_t)(kmax * d));
  double* S = buf.alloc<double>(kMaxSub * kMaxSub);
  double* y = buf.alloc<double>(kMaxSub);
  double* x = buf.alloc<double>((size_t)d);
  double* wx = buf.alloc<double>((size_t)d);
  double* r = buf.alloc<double>((size_t)d);
  double* t = buf.alloc<double>((size_t)d);
  const unsigned gd = blocks_of(d, 256), gm = blocks_of(d, 4);
  int k = 0;
  auto add_vector = [&]() -> double {   // t -> V[k] (orthonormalised), W[k] = M V[k], S column k
    hipLaunchKernelGGL(orth_append_kernel, dim3(1), dim3(256), 0, st, d, k, V, t, V + (long long)k * d, scal);
    double nrm = 0;
    CCHECK(hipMemcpyAsync(&nrm, scal + 2, 8, hipMemcpyDeviceToHost, st));
    CCHECK(hipStreamSynchronize(st));
    return nrm;
  };
  auto expand = [&]() {
    hipLaunchKernelGGL(gemv_kernel, dim3(gm), dim3(256), 0, st, d, mat, V + (long long)k * d, W + (long long)k * d);
    hipLaunchKernelGGL(dots_kernel, dim3(k + 1), dim3(256), 0, st, d, k, kMaxSub, V, W, S);
    ++k;
  };
  for (auto& g : guesses) {
    if (k == kmax) break;
    CCHECK(hipMemcpyAsync(t, g.data(), d * 8, hipMemcpyHostToDevice, st));
    if (add_vector() > 1e-8) expand();
  }
  double theta = 0, res = INFINITY;
  int it = 0;
  for (; it < kMaxIter; ++it) {
    hipLaunchKernelGGL(jacobi_lowest_kernel, dim3(1), dim3(64), 0, st, k, kMaxSub, S, y, scal);
    hipLaunchKernelGGL(ritz_kernel, dim3(gd), dim3(256), 0, st, d, k, V, W, y, scal, x, wx, r);
    hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, st, d, r, scal);
    CCHECK(hipGetLastError());
    double h[2];
    CCHECK(hipMemcpyAsync(h, scal, 16, hipMemcpyDeviceToHost, st));
    CCHECK(hipStreamSynchronize(st));
    theta = h[0];
    res = std::sqrt(std::max(h[1], 0.0));
    if (res <= kResTol || k == d) break;
    if (k == kmax) {
      // restart from the current Ritz vector
      CCHECK(hipMemcpyAsync(V, x, d * 8, hipMemcpyDeviceToDevice, st));
      CCHECK(hipMemcpyAsync(W, wx, d * 8, hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(dots_kernel, dim3(1), dim3(256), 0, st, d, 0, kMaxSub, V, W, S);
      k = 1;
    }
    hipLaunchKernelGGL(precond_kernel, dim3(gd), dim3(256), 0, st, d, r, dg, scal, t);
    if (add_vector() <= 1e-14) break;   // no new direction
    expand();
  }
  out.lambda = theta;
  out.residual = res;
  out.iterations = it + 1;
  out.converged = res <= kResTol || k == d;
  if (want_ci) {
    out.ci.resize((size_t)d);
    CCHECK(hipMemcpyAsync(out.ci.data(), x, d * 8, hipMemcpyDeviceToHost, st));
    CCHECK(hipStreamSynchronize(st));
    // phase: positive overlap with the guess, else a positive largest component
    double ov = 0;
    if (in.ci_guess)
      for (long long j = 0; j < d; ++j) ov += in.ci_guess[j] * out.ci[j];
    if (ov == 0) {
      long long m = 0;
      for (long long j = 1; j < d; ++j)
        if (std::fabs(out.ci[j]) > std::fabs(out.ci[m])) m = j;
      ov = out.ci[m];
    }
    if (ov < 0)
      for (auto& v : out.ci) v = -v;
  }
  CCHECK(hipStreamSynchronize(st));
}

}  // namespace dsrg_cas
