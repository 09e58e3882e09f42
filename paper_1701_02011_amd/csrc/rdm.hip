// Reference densities from a CAS vector, the step before the path (Sec. II.A: the method
// takes the reference through its one-, two- and three-body densities).
//
// |Psi> = sum_IJ c[I][J] |I_alpha J_beta> over alpha strings I and beta strings J (all
// n_alpha- and n_beta-subsets of the nA active orbitals, lexicographic order), a
// determinant being the alpha creators then the beta creators in ascending order on the
// vacuum (alpha spin orbitals below beta ones).  For every order k and number m of alpha
// indices, the (N - k)-electron vectors w_T = a_{t_k} ... a_{t_1} |Psi> of the ordered
// tuples T = (t_1 < ... < t_k) (m alpha then k - m beta orbitals) are gathered from c with
// the signs of the annihilations, and the densities of the spin block are their Gram
// matrix, <Psi| a+_{p_1} .. a+_{p_k} a_{q_k} .. a_{q_1} |Psi> = <w_P | w_Q>, one FP64
// contraction on the GETT kernel; a last kernel spreads it over all index orders with the
// permutation signs into the library's input layout.
#include "../../include/dsrg.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <stdexcept>
#include <string>
#include <vector>

namespace dsrg {
void set_last_error(const char* m);
}

namespace dsrg_rdm {

struct Err : std::runtime_error {
  int code;
  Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
#define RCHECK(x)                                                                            \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) {                                                                  \
      (void)hipGetLastError();                                                               \
      throw Err(e_ == hipErrorOutOfMemory ? DSRG_E_OOM : DSRG_E_HIP,                         \
                std::string(#x) + ": " + hipGetErrorString(e_));                            \
    }                                                                                        \
  } while (0)

// k-subsets of n orbitals as bit masks, lexicographic order of the sorted index lists
static std::vector<uint32_t> subsets(int n, int k) {
  std::vector<uint32_t> out;
  if (k < 0 || k > n) return out;
  std::vector<int> idx(k);
  for (int i = 0; i < k; ++i) idx[i] = i;
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

static int popc(uint32_t x) { return __builtin_popcount(x); }

// Entry (tuple t, residual string r): the source string's position in the full string
// list and the sign of annihilating the tuple's orbitals (ascending) from it, with
// `below` more electrons under every orbital of this spin (the alpha electrons for beta
// annihilations); -1 when the tuple and the residual overlap.
struct Gat {
  int src;
  int sign;
};
static std::vector<Gat> gather_table(int n, const std::vector<uint32_t>& tuples, const std::vector<uint32_t>& resid,
                                     const std::vector<int>& pos, int below) {
  std::vector<Gat> t(tuples.size() * resid.size());
  for (size_t a = 0; a < tuples.size(); ++a)
    for (size_t r = 0; r < resid.size(); ++r) {
      Gat& g = t[a * resid.size() + r];
      if (tuples[a] & resid[r]) {
        g = {-1, 0};
        continue;
      }
      uint32_t cur = tuples[a] | resid[r];
      int sgn = 1;
      for (int p = 0; p < n; ++p)
        if (tuples[a] >> p & 1u) {
          if ((popc(cur & ((1u << p) - 1u)) + below) & 1) sgn = -sgn;
          cur &= ~(1u << p);
        }
      g = {pos[tuples[a] | resid[r]], sgn};
    }
  return t;
}

// W[ta * nTb + tb][ra * nRb + rb] = c[src_a][src_b] * sign_a * sign_b
__global__ __launch_bounds__(256) void rdm_gather_kernel(const double* __restrict__ c, int nJ, const Gat* __restrict__ ga,
                                                         const Gat* __restrict__ gb, int nTa, int nTb, int nRa, int nRb,
                                                         double* __restrict__ W) {
  const long long states = (long long)nRa * nRb;
  const long long total = (long long)nTa * nTb * states;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const long long row = e / states, col = e - row * states;
    const int ta = (int)(row / nTb), tb = (int)(row - (long long)ta * nTb);
    const int ra = (int)(col / nRb), rb = (int)(col - (long long)ra * nRb);
    const Gat A = ga[(long long)ta * nRa + ra], Bt = gb[(long long)tb * nRb + rb];
    W[e] = (A.src < 0 || Bt.src < 0) ? 0.0 : c[(long long)A.src * nJ + Bt.src] * (double)(A.sign * Bt.sign);
  }
}

// Spin block with m alpha indices of order k: out[u_1..u_k][x_1..x_k] from the Gram matrix
// G[(alpha tuple, beta tuple)][(alpha tuple, beta tuple)]; rank[mask] is a subset's
// position among the subsets of its size.
__global__ __launch_bounds__(256) void rdm_expand_kernel(const double* __restrict__ G, int nA, int k, int m, int nTb,
                                                         int nT, const int* __restrict__ rank, double* __restrict__ out) {
  long long total = 1;
  for (int i = 0; i < 2 * k; ++i) total *= nA;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    int idx[6];
    long long q = e;
    for (int i = 2 * k - 1; i >= 0; --i) {
      idx[i] = (int)(q % nA);
      q /= nA;
    }
    // upper u (idx[0..k)) and lower x (idx[k..2k)): alpha part first, then beta part;
    // each part must hold distinct orbitals; sign of sorting each part
    int sign = 1, row[2], col[2];
    bool zero = false;
    for (int side = 0; side < 2 && !zero; ++side) {
      const int* v = idx + side * k;
      for (int part = 0; part < 2 && !zero; ++part) {
        const int lo = part ? m : 0, hi = part ? k : m;
        uint32_t mask = 0;
        for (int a = lo; a < hi; ++a) {
          if (mask >> v[a] & 1u) zero = true;
          mask |= 1u << v[a];
          for (int b = a + 1; b < hi; ++b)
            if (v[a] > v[b]) sign = -sign;
        }
        (side ? col : row)[part] = rank[mask];
      }
    }
    out[e] = zero ? 0.0 : sign * G[(long long)(row[0] * nTb + row[1]) * nT + (col[0] * nTb + col[1])];
  }
}

static unsigned grid_of(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 16384); }

struct Buf {
  hipStream_t st = nullptr;   // work on it is finished before the buffers are freed
  std::vector<void*> v;
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    RCHECK(hipMalloc(&p, std::max<size_t>(1, n) * sizeof(T)));
    v.push_back(p);
    return (T*)p;
  }
  ~Buf() {
    (void)hipStreamSynchronize(st);
    for (void* p : v) (void)hipFree(p);
  }
};

static long long ipow(long long b, int e) {
  long long r = 1;
  while (e-- > 0) r *= b;
  return r;
}

static void run(const double* ci, int nA, int na, int nb, const dsrg_options* O, double* g1, double* g2,
                double* g3) {
  if (nA < 1 || nA > 16) throw Err(DSRG_E_UNSUPPORTED, "active spaces of 1 to 16 orbitals");
  if (na < 0 || nb < 0 || na > nA || nb > nA) throw Err(DSRG_E_ARG, "electron counts outside 0..nA");
  if (!ci || !g1 || !g2) throw Err(DSRG_E_ARG, "null ci, gamma1 or gamma2");
  const bool dev = O && (O->flags & DSRG_F_DEVICE_PTRS);
  hipStream_t st = (O && O->stream) ? (hipStream_t)O->stream : (hipStream_t)0;
  dsrg::set_big_tile_min(0);   // the built-in tile choice (tile rules are keyed by orbital spaces)
  const std::vector<uint32_t> Sa = subsets(nA, na), Sb = subsets(nA, nb);
  const long long nI = (long long)Sa.size(), nJ = (long long)Sb.size();
  std::vector<int> pos(1u << nA, -1), rank(1u << nA, 0);
  for (int k = 0; k <= nA; ++k) {
    const std::vector<uint32_t> s = subsets(nA, k);
    for (size_t i = 0; i < s.size(); ++i) rank[s[i]] = (int)i;
  }
  Buf buf;
  buf.st = st;
  // the CI vector on the device (a copy; checked for finite values on the host path)
  double* c = buf.alloc<double>((size_t)(nI * nJ));
  if (dev) {
    RCHECK(hipMemcpyAsync(c, ci, nI * nJ * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    for (long long i = 0; i < nI * nJ; ++i)
      if (!std::isfinite(ci[i])) throw Err(DSRG_E_NONFINITE, "non-finite CI coefficient");
    RCHECK(hipMemcpyAsync(c, ci, nI * nJ * sizeof(double), hipMemcpyHostToDevice, st));
  }
  int* d_rank = buf.alloc<int>(rank.size());
  RCHECK(hipMemcpyAsync(d_rank, rank.data(), rank.size() * sizeof(int), hipMemcpyHostToDevice, st));
  std::deque<std::vector<Gat>> hold;   // host tables live until the synchronisation (a deque:
                                       // references to earlier tables stay valid)
  double* outs[3] = {g1, g2, g3};
  for (int k = 1; k <= 3; ++k) {
    if (!outs[k - 1]) continue;
    const long long blk = ipow(nA, 2 * k);
    double* dst = outs[k - 1];
    std::vector<double> host_out;
    double* d_out = dst;
    if (!dev) d_out = buf.alloc<double>((size_t)(blk * (k + 1)));
    for (int m = k; m >= 0; --m) {   // blocks in input order: all alpha first
      double* ob = d_out + (long long)(k - m) * blk;
      const std::vector<uint32_t> Ta = subsets(nA, m), Tb = subsets(nA, k - m);
      const std::vector<uint32_t> Ra = subsets(nA, na - m), Rb = subsets(nA, nb - (k - m));
      if (Ta.empty() || Tb.empty() || Ra.empty() || Rb.empty()) {
        dsrg::launch_fill(ob, blk, 0.0, st);
        continue;
      }
      std::fill(pos.begin(), pos.end(), -1);
      for (size_t i = 0; i < Sa.size(); ++i) pos[Sa[i]] = (int)i;
      hold.push_back(gather_table(nA, Ta, Ra, pos, 0));
      const std::vector<Gat>& ta = hold.back();
      std::fill(pos.begin(), pos.end(), -1);
      for (size_t i = 0; i < Sb.size(); ++i) pos[Sb[i]] = (int)i;
      hold.push_back(gather_table(nA, Tb, Rb, pos, na - m));
      const std::vector<Gat>& tb = hold.back();
      Gat* d_ta = buf.alloc<Gat>(ta.size());
      Gat* d_tb = buf.alloc<Gat>(tb.size());
      RCHECK(hipMemcpyAsync(d_ta, ta.data(), ta.size() * sizeof(Gat), hipMemcpyHostToDevice, st));
      RCHECK(hipMemcpyAsync(d_tb, tb.data(), tb.size() * sizeof(Gat), hipMemcpyHostToDevice, st));
      const long long nT = (long long)Ta.size() * Tb.size(), nS = (long long)Ra.size() * Rb.size();
      if (nT >= (1LL << 31) || nS >= (1LL << 31) || nT * nS > (1LL << 30))
        throw Err(DSRG_E_OOM, "active space too large for the one-pass density build");
      double* W = buf.alloc<double>((size_t)(nT * nS));
      hipLaunchKernelGGL(rdm_gather_kernel, dim3(grid_of(nT * nS)), dim3(256), 0, st, c, (int)nJ, d_ta, d_tb,
                         (int)Ta.size(), (int)Tb.size(), (int)Ra.size(), (int)Rb.size(), W);
      // Gram matrix G = W W^T on the GETT kernel (FP64 MFMA)
      double* G = buf.alloc<double>((size_t)(nT * nT));
      dsrg::GettDesc g;
      g.nm = 1; g.nn = 1; g.nk = 1;
      g.md[0] = (int)nT; g.nd[0] = (int)nT; g.kd[0] = (int)nS;
      g.am[0] = nS; g.ak[0] = 1; g.bk[0] = 1; g.bn[0] = nS;
      g.cm[0] = nT; g.cn[0] = 1;
      g.M = (int)nT; g.N = (int)nT; g.K = (int)nS;
      g.alpha = 1.0; g.beta = 0;
      dsrg::gett_prepare(g);
      dsrg::launch_gett(g, W, W, G, st, dsrg::kRoleGeneric, nullptr, 0, 0);
      hipLaunchKernelGGL(rdm_expand_kernel, dim3(grid_of(blk)), dim3(256), 0, st, G, nA, k, m, (int)Tb.size(),
                         (int)nT, d_rank, ob);
      RCHECK(hipGetLastError());
    }
    if (!dev) RCHECK(hipMemcpyAsync(dst, d_out, blk * (k + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  RCHECK(hipStreamSynchronize(st));
  RCHECK(hipGetLastError());
}

}  // namespace dsrg_rdm

extern "C" int dsrg_active_rdms(const double* ci, int32_t n_active, int32_t n_alpha, int32_t n_beta,
                                const dsrg_options* opt, double* gamma1, double* gamma2, double* gamma3) {
  try {
    dsrg_rdm::run(ci, n_active, n_alpha, n_beta, opt, gamma1, gamma2, gamma3);
    dsrg::set_last_error("");
    return DSRG_OK;
  } catch (const dsrg_rdm::Err& e) {
    dsrg::set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    dsrg::set_last_error(e.what());
    return DSRG_E_HIP;
  }
}
