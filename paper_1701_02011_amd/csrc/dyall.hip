// Active-to-virtual doubles under Dyall's zeroth-order Hamiltonian (App. B, Eq. t2_aavv).
//
// With the active two-body interaction in H0 and s -> inf, the amplitudes t_{ef}^{uv} of
// one virtual pair (e, f) solve
//     (Delta_{ef}^{uv}) t^{uv} + 1/2 sum_{xy} v_{xy}^{uv} t^{xy} - sum_{xyz} v_{xy}^{uv} t^{xz} gamma_z^y = v_{ef}^{uv}
// with Delta_{ef}^{uv} = e_u + e_v - e_e - e_f.  The coupling K does not depend on (e, f);
// the pair enters only through the shift e_e + e_f on the diagonal.  The paper solves
// the coupled amplitudes iteratively; here the system is block diagonal over virtual pairs
// and spin blocks, so every block (at most nA^2 unknowns) is solved exactly by Gaussian
// elimination in LDS, one workgroup per block, all blocks in one launch.
//
// Spin blocks (restricted orbitals, gamma^alpha and gamma^beta distinct):
//   aa: K[(uv),(ab)] = v0(a,b,u,v) - sum_y [v0(a,y,u,v) ga(y,b) - v0(b,y,u,v) ga(y,a)]
//       over unique pairs u < v, a < b, with v0(x,y,u,v) = (xu|yv) - (xv|yu);
//   ab: K[(uv),(ab)] = (au|bv) - sum_y (au|yv) gb(y,b) - sum_y (bv|yu) ga(y,a)
//       over ordered (u alpha, v beta), (a alpha, b beta);
//   bb: as aa with gb.
// The right-hand sides are <ef||uv>: (eu|fv) - (ev|fu) (aa, bb) and (eu|fv) (ab).
#include "dyall.h"

#include <cmath>

namespace dsrg_dyall {

__device__ __forceinline__ double jget(const double* J, int n, int x, int u, int y, int v) {
  return J[(((long long)x * n + u) * n + y) * n + v];
}

// unique pair index of u < v among n indices (row-major)
__device__ __forceinline__ int pair_index(int n, int u, int v) { return u * n - u * (u + 1) / 2 + (v - u - 1); }

__global__ void operator_kernel(int nA, const double* __restrict__ J, const double* __restrict__ g1,
                                double* __restrict__ Kaa, double* __restrict__ Kbb, double* __restrict__ Kab) {
  const int np = nA * (nA - 1) / 2, n2 = nA * nA;
  const long long naa = (long long)np * np, nab = (long long)n2 * n2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double* ga = g1;
  const double* gb = g1 + n2;
  if (idx < nab) {
    const int r = (int)(idx / n2), c = (int)(idx % n2);
    const int u = r / nA, v = r % nA, a = c / nA, b = c % nA;
    double s = jget(J, nA, a, u, b, v);
    for (int y = 0; y < nA; ++y)
      s -= jget(J, nA, a, u, y, v) * gb[y * nA + b] + jget(J, nA, b, v, y, u) * ga[y * nA + a];
    Kab[idx] = s;
    return;
  }
  long long k = idx - nab;
  if (k >= 2 * naa) return;
  const int spin = (int)(k / naa);
  k -= spin * naa;
  const double* g = spin ? gb : ga;
  const int r = (int)(k / np), c = (int)(k % np);
  // pair r -> (u, v), c -> (a, b)
  int u = 0, rr = r;
  while (rr >= nA - 1 - u) {
    rr -= nA - 1 - u;
    ++u;
  }
  const int v = u + 1 + rr;
  int a = 0, cc = c;
  while (cc >= nA - 1 - a) {
    cc -= nA - 1 - a;
    ++a;
  }
  const int b = a + 1 + cc;
  auto v0 = [&](int x, int y) { return jget(J, nA, x, u, y, v) - jget(J, nA, x, v, y, u); };
  double s = v0(a, b);
  for (int y = 0; y < nA; ++y) s -= v0(a, y) * g[y * nA + b] - v0(b, y) * g[y * nA + a];
  (spin ? Kbb : Kaa)[k] = s;
}

void launch_operator(int nA, const double* Jaaaa, const double* g1, double* Kaa, double* Kbb,
                     double* Kab, hipStream_t st) {
  const long long np = (long long)nA * (nA - 1) / 2, n2 = (long long)nA * nA;
  const long long total = n2 * n2 + 2 * np * np;
  if (total == 0) return;
  hipLaunchKernelGGL(operator_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, nA, Jaaaa, g1,
                     Kaa, Kbb, Kab);
}

// Workgroup (blockIdx.x = e * nV + f, blockIdx.y = spin block 0 aa, 1 ab, 2 bb).  The same-
// spin blocks are solved for e < f only; that workgroup also writes the mirrored slab
// t[f][e] = -t[e][f], and the e == f workgroup writes zeros.
__global__ __launch_bounds__(256) void solve_kernel(int nC, int nA, int nV, const double* __restrict__ eps,
                                                    const double* __restrict__ J, const double* __restrict__ Kaa,
                                                    const double* __restrict__ Kbb, const double* __restrict__ Kab,
                                                    double* __restrict__ t, double* __restrict__ dmin,
                                                    int* __restrict__ singular) {
  extern __shared__ double sm[];
  __shared__ int piv, sing;
  __shared__ double red[4];
  const int kind = blockIdx.y;
  const int e = blockIdx.x / nV, f = blockIdx.x % nV;
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const long long slab = (long long)nA * nA;
  double* tb = t + (long long)kind * nV * nV * slab;
  double* out = tb + ((long long)e * nV + f) * slab;
  const long long sys = (long long)kind * nV * nV + blockIdx.x;
  const bool same = kind != 1;
  const int n = same ? nA * (nA - 1) / 2 : nA * nA;
  if (n == 0 || (same && e >= f)) {
    // no unknowns (a same-spin block of one active orbital) or the e == f slab: zeros; the
    // e > f slabs of the same-spin blocks are written by their e < f workgroup
    if (n == 0 || e == f)
      for (long long k = tid; k < slab; k += bs) out[k] = 0.0;
    if (tid == 0) dmin[sys] = INFINITY;
    return;
  }
  const int ld = n + 1;
  const double* K = kind == 0 ? Kaa : kind == 1 ? Kab : Kbb;
  const double se = eps[nC + nA + e] + eps[nC + nA + f];
  const double* ea = eps + nC;
  // decode of row i: (u, v)
  auto uv = [&](int i, int& u, int& v) {
    if (!same) {
      u = i / nA;
      v = i - u * nA;
      return;
    }
    int uu = 0, r = i;
    while (r >= nA - 1 - uu) {
      r -= nA - 1 - uu;
      ++uu;
    }
    u = uu;
    v = uu + 1 + r;
  };
  // load [Delta + K | v] and the scale of the block
  double amax = 0.0, dm = INFINITY;
  for (int idx = tid; idx < n * ld; idx += bs) {
    const int i = idx / ld, j = idx - i * ld;
    int u, v;
    uv(i, u, v);
    double x;
    if (j == n) {
      const double c = J[(((long long)e * nA + u) * nV + f) * nA + v];
      x = same ? c - J[(((long long)e * nA + v) * nV + f) * nA + u] : c;
    } else {
      x = K[(long long)i * n + j];
      if (i == j) {
        x += ea[u] + ea[v] - se;
        dm = fmin(dm, fabs(x));
      }
      amax = fmax(amax, fabs(x));
    }
    sm[idx] = x;
  }
  for (int w = 32; w > 0; w >>= 1) {
    amax = fmax(amax, __shfl_xor(amax, w, 64));
    dm = fmin(dm, __shfl_xor(dm, w, 64));
  }
  if (lane == 0) {
    red[wave] = amax;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0;
    for (int w = 0; w < bs / 64; ++w) a = fmax(a, red[w]);
    red[0] = a;
    sing = 0;
  }
  // block minimum of |diagonal| through the LDS slot of each wave (after the barrier above)
  __syncthreads();
  const double tol = 1e-13 * red[0];
  __syncthreads();
  if (lane == 0) red[wave] = dm;
  __syncthreads();
  if (tid == 0) {
    double d = INFINITY;
    for (int w = 0; w < bs / 64; ++w) d = fmin(d, red[w]);
    dmin[sys] = d;
  }
  // Gaussian elimination with partial pivoting on the augmented matrix
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = k;
      for (int i = k + lane; i < n; i += 64) {
        const double a = fabs(sm[i * ld + k]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      for (int w = 32; w > 0; w >>= 1) {
        const double ob = __shfl_xor(best, w, 64);
        const int oi = __shfl_xor(bi, w, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        piv = bi;
        if (!(best > tol)) sing = 1;
      }
    }
    __syncthreads();
    if (sing) break;   // uniform: read after the barrier
    const int p = piv;
    if (p != k)
      for (int j = k + tid; j <= n; j += bs) {
        const double a = sm[k * ld + j];
        sm[k * ld + j] = sm[p * ld + j];
        sm[p * ld + j] = a;
      }
    __syncthreads();
    const double pk = sm[k * ld + k];
    for (int i = k + 1 + tid; i < n; i += bs) sm[i * ld + k] /= pk;
    __syncthreads();
    const int rows = n - k - 1, cols = n - k;
    for (int idx = tid; idx < rows * cols; idx += bs) {
      const int i = k + 1 + idx / cols, j = k + 1 + idx % cols;
      sm[i * ld + j] -= sm[i * ld + k] * sm[k * ld + j];
    }
    __syncthreads();
  }
  if (sing) {
    if (tid == 0) atomicOr(singular, 1);
    for (long long k = tid; k < slab; k += bs) {
      out[k] = NAN;
      if (same) tb[((long long)f * nV + e) * slab + k] = NAN;
    }
    return;
  }
  // back substitution: x_k into column n
  for (int k = n - 1; k >= 0; --k) {
    if (tid == 0) sm[k * ld + n] /= sm[k * ld + k];
    __syncthreads();
    const double xk = sm[k * ld + n];
    for (int i = tid; i < k; i += bs) sm[i * ld + n] -= sm[i * ld + k] * xk;
    __syncthreads();
  }
  if (!same) {
    for (int i = tid; i < n; i += bs) out[i] = sm[i * ld + n];
    return;
  }
  double* mir = tb + ((long long)f * nV + e) * slab;
  for (int k = tid; k < nA * nA; k += bs) {
    const int u = k / nA, v = k - u * nA;
    double x = 0.0;
    if (u < v) x = sm[pair_index(nA, u, v) * ld + n];
    else if (u > v) x = -sm[pair_index(nA, v, u) * ld + n];
    out[k] = x;
    mir[k] = -x;
  }
}

void launch_solve(int nC, int nA, int nV, const double* eps, const double* Jvava, const double* Kaa,
                  const double* Kbb, const double* Kab, double* t, double* dmin, int* singular,
                  hipStream_t st) {
  if (nV == 0 || nA == 0) return;
  const int n = nA * nA;
  const size_t lds = (size_t)n * (n + 1) * sizeof(double);
  hipLaunchKernelGGL(solve_kernel, dim3((unsigned)nV * nV, 3), dim3(256), lds, st, nC, nA, nV, eps, Jvava,
                     Kaa, Kbb, Kab, t, dmin, singular);
}

__global__ void min_kernel(const double* __restrict__ x, long long n, double* __restrict__ out) {
  __shared__ double red[4];
  double m = INFINITY;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) m = fmin(m, x[i]);
  for (int w = 32; w > 0; w >>= 1) m = fmin(m, __shfl_xor(m, w, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = INFINITY;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) r = fmin(r, red[w]);
    out[0] = r;
  }
}

void launch_min(const double* dmin, long long n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(min_kernel, dim3(1), dim3(256), 0, st, dmin, n, out);
}

}  // namespace dsrg_dyall
