// DSRG-MRPT3 hot path on one MI355X: C ABI, contraction-table executor and pipeline.
//
// The steps follow Sec. II.B of the paper: first-order amplitudes (Eqs. T1_1st, T2_1st),
// E(2) = <[H~(1), T(1)]>, O1 = [H~(1), A(1)]_{1,2} with H~(1) = 2 V + Y and
// Y = [H(0), A(1)] (so O1 = 2 [V, A(1)] + [Y, A(1)]), second-order amplitudes from the
// non-diagonal part of O1/2 (Eqs. T1_2nd, T2_2nd), H~(2)_{1,2} = [H(0), A(2)] + O1/2 - [Y, A(1)]/6
// and E(3) = <[H~(1), T(2)]> + <[H~(2)_{1,2}, T(1)]>.  The commutator terms come from the
// generated table in dsrg_terms.inc; every contraction in it runs on the GETT kernel.
#include "../../include/dsrg.h"
#include "../../include/dsrg_testing.h"
#include "cas.h"
#include "dyall.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "dsrg_terms.inc"

namespace dsrg {

static thread_local std::string g_last_error;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHECK(x)                                                                          \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) {                                                                  \
      if (e_ == hipErrorOutOfMemory) throw Error(DSRG_E_OOM, std::string(#x) + ": out of memory"); \
      throw Error(DSRG_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));               \
    }                                                                                        \
  } while (0)

// ---------------------------------------------------------------------------
// Orbital spaces: C, A, V, H = C+A, P = A+V, G; contiguous in [C|A|V] order
// ---------------------------------------------------------------------------
struct Dims {
  int nC, nA, nV;
  int off(char s) const {
    switch (s) {
      case 'C': case 'H': case 'G': return 0;
      case 'A': case 'P': return nC;
      case 'V': return nC + nA;
    }
    throw Error(DSRG_E_ARG, "bad space");
  }
  int len(char s) const {
    switch (s) {
      case 'C': return nC;
      case 'A': return nA;
      case 'V': return nV;
      case 'H': return nC + nA;
      case 'P': return nA + nV;
      case 'G': return nC + nA + nV;
    }
    throw Error(DSRG_E_ARG, "bad space");
  }
};

// ---------------------------------------------------------------------------
// Contraction table
// ---------------------------------------------------------------------------
struct TFactor {
  std::string tensor, block, letters;
};
struct TScatter {
  double coef;
  std::string tensor, block, letters;
};
struct TProduct {
  std::vector<TFactor> f;
  std::map<char, char> space;
  std::string res;
  std::vector<TScatter> s;
};
using Use = std::vector<TProduct>;

static std::map<std::string, Use>& table() {
  static std::map<std::string, Use> t;
  static std::once_flag once;
  std::call_once(once, [] {
    std::istringstream in(kDsrgTermTable);
    std::string line;
    Use* cur = nullptr;
    while (std::getline(in, line)) {
      if (line.empty()) continue;
      std::istringstream ls(line);
      std::string tag;
      ls >> tag;
      if (tag == "U") {
        std::string name;
        ls >> name;
        cur = &t[name];
      } else if (tag == "P") {
        TProduct p;
        int nf;
        ls >> nf;
        for (int i = 0; i < nf; ++i) {
          std::string tok;
          ls >> tok;
          size_t dot = tok.find('.'), col = tok.find(':');
          TFactor f{tok.substr(0, dot), tok.substr(dot + 1, col - dot - 1), tok.substr(col + 1)};
          if (f.block == "-") f.block = "";
          p.f.push_back(f);
        }
        std::string bar;
        ls >> bar;  // '|'
        std::string tok;
        while (ls >> tok && tok != "|") p.space[tok[0]] = tok[2];
        ls >> p.res;
        if (p.res == "-") p.res = "";
        cur->push_back(p);
      } else if (tag == "S") {
        TScatter s;
        std::string tgt;
        ls >> s.coef >> tgt;
        size_t dot = tgt.find('.'), col = tgt.find(':');
        s.tensor = tgt.substr(0, dot);
        s.block = tgt.substr(dot + 1, col - dot - 1);
        s.letters = tgt.substr(col + 1);
        if (s.block == "-") s.block = "";
        if (s.letters == "-") s.letters = "";
        cur->back().s.push_back(s);
      }
    }
  });
  return t;
}

// Gradient of the scalar use C0 with respect to its doubles factor, restricted to core
// holes: E(3) is linear in the amplitudes of its final commutators, so each C0 product
// with a doubles factor T2[a,b,i,j] becomes the product of its other factors with the free
// letters a,b,i,j (each of them appears in exactly one other factor), scattered into
// G2.<block>; the hole letters run over the core only.  sum_ab G2[a,b,i,j] T2[a,b,i,j]
// is then the contribution of the core pair's amplitudes.  Products with a singles
// factor, or whose doubles factor has an active-only hole letter, belong to the rest.
static const Use& pair_use() {
  static Use u;
  static std::once_flag once;
  std::call_once(once, [] {
    for (const TProduct& P : table().at("C0")) {
      int t2 = -1, t1 = -1;
      for (size_t k = 0; k < P.f.size(); ++k) {
        if (P.f[k].tensor == "T2") t2 = (int)k;
        if (P.f[k].tensor == "T1") t1 = (int)k;
      }
      if (t1 >= 0 || t2 < 0) continue;
      const TFactor T = P.f[t2];   // storage [P][P][H][H]
      TProduct Q = P;
      bool active_hole = false;
      for (int k = 2; k < 4; ++k) {
        char& sp = Q.space.at(T.letters[k]);
        if (sp == 'A') active_hole = true;
        sp = 'C';
      }
      if (active_hole) continue;
      Q.f.erase(Q.f.begin() + t2);
      double coef = 0;
      for (auto& sc : P.s) coef += sc.coef;
      Q.res = T.letters;
      Q.s.clear();
      Q.s.push_back(TScatter{coef, "G2", T.block, T.letters});
      u.push_back(Q);
    }
  });
  return u;
}

// A commutator use restricted to the two-body outputs whose hole pair has at least one
// active index (and all one-body outputs): in every product that writes the two-body
// excitation block, each hole letter of the output (third and fourth output letters of its
// scatters) that runs over all holes is split into its core and active parts, and the
// core-core combination is dropped.  With these uses the second-order amplitudes vanish on
// core-core hole pairs, which is what the rest of the core-pair decomposition of E(3)
// needs (the scalars pair the hole indices of the two operators within one space).
static Use rest_use(const Use& U) {
  Use out;
  for (const TProduct& P : U) {
    std::string holes;
    for (auto& sc : P.s)
      if (sc.letters.size() == 4)
        for (int k = 2; k < 4; ++k)
          if (holes.find(sc.letters[k]) == std::string::npos) holes += sc.letters[k];
    if (holes.empty()) {
      out.push_back(P);
      continue;
    }
    std::vector<std::vector<char>> opt;
    for (char l : holes) {
      const char sp = P.space.at(l);
      if (sp == 'H') opt.push_back({'C', 'A'});
      else opt.push_back({sp});
    }
    std::vector<size_t> pick(opt.size(), 0);
    while (true) {
      bool all_core = true;
      TProduct Q = P;
      for (size_t k = 0; k < opt.size(); ++k) {
        Q.space[holes[k]] = opt[k][pick[k]];
        all_core = all_core && opt[k][pick[k]] == 'C';
      }
      if (!all_core) out.push_back(Q);
      size_t k = 0;
      while (k < opt.size() && ++pick[k] == opt[k].size()) pick[k++] = 0;
      if (k == opt.size()) break;
    }
  }
  return out;
}

static const char* storage_axes(const std::string& t) {
  if (t == "T1" || t == "E1" || t == "Y1" || t == "O1" || t == "F1") return "PH";
  if (t == "T2" || t == "E2" || t == "Y2" || t == "O2") return "PPHH";
  if (t == "L2") return "AAAA";
  if (t == "L3") return "AAAAAA";
  if (t == "gA" || t == "eA") return "AA";
  throw Error(DSRG_E_ARG, "unknown tensor " + t);
}

// ---------------------------------------------------------------------------
// Device memory.  A call-scoped pool frees its buffers when the call ends; a plan-owned
// pool (keep = true) never frees before the plan is destroyed, because a captured graph
// addresses every buffer of the pipeline.
// ---------------------------------------------------------------------------
// Large device buffers kept across calls.  Allocating and freeing tens of GB per call
// (the resident (PP|PP) block, its packed rows) made later calls of the same process stall
// for seconds inside the runtime; a buffer of at least kBigBytes goes back to this list
// when its pool is destroyed (its work finished: the pool synchronises its stream, or a
// plan's last use did) and serves a later request of the same device that it covers
// within a factor of two.  At most kCachedBytes stay listed; dsrg_release_cache() and a
// failed allocation empty the list.
constexpr size_t kBigBytes = 64ULL << 20;
constexpr size_t kCachedBytes = 96ULL << 30;
struct BigCache {
  std::mutex mu;
  struct Buf {
    int dev;
    size_t bytes;
    void* p;
  };
  std::vector<Buf> free_list;
  size_t held = 0;
  // a listed buffer of dev holding at least `bytes` (and at most twice that), or null;
  // *got receives its size
  void* take(int dev, size_t bytes, size_t* got) {
    std::lock_guard<std::mutex> lk(mu);
    int best = -1;
    for (int i = 0; i < (int)free_list.size(); ++i) {
      const Buf& b = free_list[i];
      if (b.dev == dev && b.bytes >= bytes && b.bytes <= 2 * bytes &&
          (best < 0 || b.bytes < free_list[best].bytes))
        best = i;
    }
    if (best < 0) return nullptr;
    void* p = free_list[best].p;
    *got = free_list[best].bytes;
    held -= free_list[best].bytes;
    free_list.erase(free_list.begin() + best);
    return p;
  }
  void give(int dev, size_t bytes, void* p) {
    std::lock_guard<std::mutex> lk(mu);
    free_list.push_back({dev, bytes, p});
    held += bytes;
    while (held > kCachedBytes && !free_list.empty()) {   // oldest first
      held -= free_list.front().bytes;
      (void)hipFree(free_list.front().p);
      free_list.erase(free_list.begin());
    }
  }
  void clear() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto& b : free_list) (void)hipFree(b.p);
    free_list.clear();
    held = 0;
  }
};
static BigCache& big_cache() {
  static BigCache* c = new BigCache;   // never destroyed: buffers outlive static teardown
  return *c;
}

struct Pool {
  hipStream_t st;     // synchronised before freeing while sync_before_free is set
  bool keep;
  bool sync_before_free = true;
  std::vector<void*> bufs;
  std::vector<size_t> sizes;   // bytes of each buffer (cached big buffers may be larger)
  int dev = -1;
  size_t bytes = 0;
  // arena mode: buffers are carved in order from [arena, arena + arena_cap) (256-byte
  // aligned) and never freed; nothing is allocated from the runtime
  char* arena = nullptr;
  size_t arena_cap = 0;
  explicit Pool(hipStream_t s, bool keep_ = false) : st(s), keep(keep_) {}
  Pool(hipStream_t s, char* base, size_t cap) : st(s), keep(true), sync_before_free(false), arena(base), arena_cap(cap) {}
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  double* alloc(size_t n) {
    if (n == 0) n = 1;
    if (arena) {
      const size_t need = (n * sizeof(double) + 255) & ~(size_t)255;
      if (bytes + need > arena_cap)
        throw Error(DSRG_E_OOM, "the problem needs more than the " + std::to_string(arena_cap >> 20) +
                                    " MiB of the static scratch (" + std::to_string(bytes + need) + " bytes so far)");
      double* p = reinterpret_cast<double*>(arena + bytes);
      bytes += need;
      return p;
    }
    void* p = nullptr;
    size_t got = n * sizeof(double);
    if (got >= kBigBytes) {
      if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(DSRG_E_HIP, "hipGetDevice failed");
      }
      p = big_cache().take(dev, got, &got);
    }
    if (!p) {
      hipError_t e = hipMalloc(&p, got);
      if (e != hipSuccess && got >= kBigBytes) {
        (void)hipGetLastError();
        big_cache().clear();
        e = hipMalloc(&p, got);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(DSRG_E_OOM, "device allocation of " + std::to_string(n * 8) + " bytes failed");
      }
    }
    bufs.push_back(p);
    sizes.push_back(got);
    bytes += n * 8;
    return (double*)p;
  }
  void release(double* p) {
    if (keep) return;
    for (auto& b : bufs)
      if (b == p) {
        (void)hipFree(b);   // synchronises with the work that may still read it
        b = nullptr;
      }
  }
  ~Pool() {
    if (sync_before_free) (void)hipStreamSynchronize(st);
    for (size_t i = 0; i < bufs.size(); ++i) {
      if (!bufs[i]) continue;
      if (sizes[i] >= kBigBytes && dev >= 0) big_cache().give(dev, sizes[i], bufs[i]);
      else (void)hipFree(bufs[i]);
    }
  }
};

// Device operations of the pipeline: each runs at once on the call's stream and, while a
// plan is being built, is also kept (by value) for capture into a HIP graph.
using DevOp = std::function<void(hipStream_t)>;
struct OpLog {
  hipStream_t st;
  std::vector<DevOp>* rec = nullptr;
  hipStream_t side = nullptr;   // set: ops of a forked branch, run on this stream
  bool defer = false;           // record only (into rec); the caller runs the list later
  void operator()(DevOp f) {
    if (defer) {
      rec->push_back(std::move(f));
      return;
    }
    if (side) {
      DevOp g = [f = std::move(f), sd = side](hipStream_t) { f(sd); };
      g(st);
      if (rec) rec->push_back(std::move(g));
      return;
    }
    f(st);
    if (rec) rec->push_back(std::move(f));
  }
};

// A strided view of a stored tensor with one letter per axis.
struct Opnd {
  const double* p;
  std::string letters;
  std::vector<long long> stride;
  long long lim = 0;   // elements addressable from p (allocation end)
  long long toff = -1; // grouped planning: offset in the temporary arena (p unset)
};

struct TensorRef {
  double* p;
  std::string axes;               // storage spaces per axis
  std::vector<long long> stride;  // element strides per axis
  long long lim = 0;              // elements addressable from p
  // known symmetry of a [P][P][H][H] doubles tensor: 1 antisymmetric in the particle pair
  // and in the hole pair; 2 T[x][y][i][j] = T[y][x][j][i]; 0 none assumed
  int sym = 0;
};

// Host-side bounds check of a strided view before any launch that reads or writes it.
static void check_view(const char* what, long long lim, const std::vector<long long>& stride,
                       const std::vector<int>& len) {
  long long hi = 0;
  for (size_t k = 0; k < stride.size(); ++k) {
    if (len[k] <= 0) return;
    if (stride[k] < 0) throw Error(DSRG_E_HIP, std::string("internal: negative stride in ") + what);
    hi += (long long)(len[k] - 1) * stride[k];
  }
  if (hi >= lim)
    throw Error(DSRG_E_HIP, std::string("internal: view of ") + what + " addresses past its allocation");
}

// ---------------------------------------------------------------------------
// Executor
// ---------------------------------------------------------------------------
struct Exec {
  Dims d;
  hipStream_t st;
  Pool& pool;
  OpLog& op;
  const double* B;   // [M][N][N] device
  int M;
  std::map<std::string, TensorRef> tensors;   // "T2.aa" -> view
  std::map<std::string, double*> jblocks;     // "HPHP" -> [X1][X2][X3][X4]
  double* partial = nullptr;
  long long ws_cap;
  int virt_batch = 0;   // requested (PP|PP) batch size (0: the largest that fits ws_cap)
  double gett_flops = 0, ladder_flops = 0, ladder_ms = 0;
  int ladder_batch = 0, n_launch = 0;

  Exec(Dims d_, hipStream_t s, Pool& p, OpLog& o, const double* B_, int M_, long long cap, bool prof)
      : d(d_), st(s), pool(p), op(o), B(B_), M(M_), ws_cap(cap), profile(prof) {
    partial = pool.alloc(dot_partials());
  }
  // split-K partial tiles, grown on demand up to kSplitCap doubles; launches on one stream
  // use the buffer in order, and a replaced buffer stays allocated until the call ends
  static constexpr long long kSplitCap = 1LL << 27;
  long long splitk_elems = 0;
  double* splitk_ws = nullptr;
  double* splitk_buffer(long long n) {
    if (n <= 0) return nullptr;
    if (n > splitk_elems) {
      splitk_ws = pool.alloc((size_t)n);
      splitk_elems = n;
    }
    return splitk_ws;
  }

  // every contraction launch goes through here; with profiling, HIP events bracket it
  bool profile;
  bool no_side = false;   // keep every launch on the caller's stream (no library stream or events)
  int role_now = kRoleGeneric;
  struct Rec {
    hipEvent_t a, b;
    int role;
    double flops;
    int M, N, K, nm, nn, nk;
    int product;
    double bytes = 0;   // algorithmic bytes: operands read once, result written once
    int big = 0;        // 128 x 128 tiles (a kernel instance of its own)
    // layout after preparation, for the per-launch dump
    int kin = 0, ksteps = 0, akf = 0, bkf = 0, pa = 0, pb = 0, splits = 1;
    long long ai = 0, bi = 0, am = 0, bn = 0;
  };
  int cur_product = -1;
  std::vector<Rec> recs;
  // Packed copies of operands that the contraction kernel would read without unit stride
  // along its fast load direction: [m][k] for A, [n][k] for B with the kernel's inner k
  // last, so both load with k fastest.  Only when the other free dimension is large
  // enough for the copy to cost a small fraction of the contraction.
  static constexpr long long kPackMin = 64, kPackCap = 1LL << 28;
  // tile block of the triangular build of the resident (PP|PP) block (a multiple of 32)
  static constexpr int kFullKBlock = 128;
  double* pack_buf[2] = {nullptr, nullptr};
  long long pack_elems[2] = {0, 0};
  static bool unit_fast(bool kfast, int nfree, const long long* free_stride, long long k_inner) {
    if (kfast) return std::llabs(k_inner) == 1;
    return nfree > 0 && std::llabs(free_stride[nfree - 1]) == 1;
  }
  const double* pack_operand(int which, GettDesc& g, const double* src) {
    const bool isA = which == 0;
    const int nf = isA ? g.nm : g.nn;
    const int* fd = isA ? g.md : g.nd;
    long long* fs = isA ? g.am : g.bn;
    long long* ks = isA ? g.ak : g.bk;
    const long long n = (long long)(isA ? g.M : g.N) * g.K;
    PackDesc pd;
    pd.n = n;
    pd.rank = nf + g.nk;
    for (int i = 0; i < nf; ++i) { pd.d[i] = fd[i]; pd.ss[i] = fs[i]; }
    for (int j = 0; j < g.nk; ++j) { pd.d[nf + j] = g.kd[j]; pd.ss[nf + j] = ks[j]; }
    if (n > pack_elems[which]) {
      pack_buf[which] = pool.alloc((size_t)n);
      pack_elems[which] = n;
    }
    double* dst = pack_buf[which];
    op([pd, src, dst](hipStream_t s) { launch_pack(pd, src, dst, s); });
    ++n_launch;
    long long st = 1;
    for (int j = g.nk - 1; j >= 0; --j) { ks[j] = st; st *= g.kd[j]; }
    for (int i = nf - 1; i >= 0; --i) { fs[i] = st; st *= fd[i]; }
    return dst;
  }

  void gett(const GettDesc& g0, const double* A, const double* Bp, double* C, int role) {
    // the split-K and packing buffers are shared by every serial contraction: one on the
    // main stream waits for an open side branch
    if (side_pending && !op.side) join_side();
    GettDesc g = g0;
    // with FP32 or BF16 x3 products, 128 x 128 tiles only from 8 k steps
    g.big_min_steps = prec != 0 ? 8 : 0;
    // A short inner k component wastes most of each zero-padded k step: packing both
    // operands makes the whole k range one contiguous component (steps of kGettBK).
    const bool padk = g.nk > 1 && gett_k_fill(g) * 9 < 8 && g.M >= kPackMin && g.N >= kPackMin &&
                      (long long)g.M * g.K <= kPackCap && (long long)g.N * g.K <= kPackCap;
    const bool pa = padk || (!unit_fast(g.a_kfast, g.nm, g.am, g.ak[g.nk - 1]) && g.N >= kPackMin &&
                             (long long)g.M * g.K <= kPackCap);
    const bool pb = padk || (!unit_fast(g.b_kfast, g.nn, g.bn, g.bk[g.nk - 1]) && g.M >= kPackMin &&
                             (long long)g.N * g.K <= kPackCap);
    if (pa) A = pack_operand(0, g, A);
    if (pb) Bp = pack_operand(1, g, Bp);
    if (pa || pb) gett_prepare(g);
    const double frac = gett_tile_fraction(g);
    double fl = 2.0 * g.M * (double)g.N * g.K * frac;
    Rec r{nullptr, nullptr, role, fl, g.M, g.N, g.K, g.nm, g.nn, g.nk, cur_product};
    r.bytes = 8.0 * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N * frac * (g.beta ? 2 : 1));
    r.kin = g.kd[g.nk - 1]; r.ksteps = g.ksteps; r.akf = g.a_kfast; r.bkf = g.b_kfast;
    r.pa = pa; r.pb = pb;
    r.ai = g.ak[g.nk - 1]; r.bi = g.bk[g.nk - 1];
    r.am = g.nm ? g.am[g.nm - 1] : 0; r.bn = g.nn ? g.bn[g.nn - 1] : 0;
    r.big = gett_big_tiles(g) ? 1 : 0;
    if (profile) {
      HIPCHECK(hipEventCreate(&r.a));
      HIPCHECK(hipEventCreate(&r.b));
      HIPCHECK(hipEventRecord(r.a, st));
    }
    const int ns = gett_splits(g, kSplitCap);
    r.splits = ns;
    const long long wse = ns > 1 ? (long long)ns * g.M * g.N : gett_tail_ws(g);
    double* ws = splitk_buffer(wse);
    const int lo = prec;
    op([g, A, Bp, C, role, ws, wse, lo](hipStream_t s) { launch_gett(g, A, Bp, C, s, role, ws, wse, lo); });
    if (profile) {
      HIPCHECK(hipEventRecord(r.b, st));
      recs.push_back(r);
    }
    gett_flops += fl;
    if (role == kRoleLadder) ladder_flops_products += fl;
    ++n_launch;
  }
  double ladder_flops_products = 0;
  // per-role totals of profiled launches: seconds, launches, flops
  double role_sec[kRoles] = {}, role_flops[kRoles] = {}, role_bytes[kRoles] = {};
  int role_n[kRoles] = {};
  // the same per kernel instance: index 2 * role + (128 x 128 tiles)
  double kern_sec[2 * kRoles] = {}, kern_flops[2 * kRoles] = {};
  int kern_n[2 * kRoles] = {};
  void collect_profile() {
    // optional per-launch dump (shape and device time) for tuning
    const char* dump = getenv("DSRG_PROFILE_DUMP");
    FILE* fd = dump ? fopen(dump, "a") : nullptr;
    for (auto& r : recs) {
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      if (fd)
        fprintf(fd, "%d,%d,%d,%d,%d,%d,%d,%d,%.6f,%d,%d,%d,%d,%d,%d,%d,%lld,%lld,%lld,%lld\n", r.product,
                r.role, r.M, r.N, r.K, r.nm, r.nn, r.nk, ms, r.kin, r.ksteps, r.akf, r.bkf, r.pa, r.pb,
                r.splits, r.ai, r.bi, r.am, r.bn);
      role_sec[r.role] += ms * 1e-3;
      role_flops[r.role] += r.flops;
      role_bytes[r.role] += r.bytes;
      role_n[r.role] += 1;
      const int kk = 2 * r.role + (r.big ? 1 : 0);
      kern_sec[kk] += ms * 1e-3;
      kern_flops[kk] += r.flops;
      kern_n[kk] += 1;
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    if (fd) fclose(fd);
    recs.clear();
  }
  ~Exec() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    // a branch left open by an error may still run: it ends before its buffers can be freed
    if (side_st) (void)hipStreamSynchronize(side_st);
    for (auto e : side_ev) (void)hipEventDestroy(e);
    if (side_st) (void)hipStreamDestroy(side_st);
  }

  // A branch beside the main sequence (the (PP|PP) ladder beside the grouped launches of
  // the same commutators): fork_side() orders it after everything recorded so far, the ops
  // recorded until end_side() run on a second stream (default priority), and join_side()
  // orders the main sequence after them.  A capture records the same fork and join as
  // graph dependencies.  The events and the stream live until the executor ends.
  hipStream_t side_st = nullptr, main_st = nullptr;
  std::vector<hipEvent_t> side_ev;
  bool side_pending = false;
  hipEvent_t side_event() {
    hipEvent_t e = nullptr;
    HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    side_ev.push_back(e);
    return e;
  }
  void fork_side() {
    if (op.side || side_pending) throw Error(DSRG_E_HIP, "internal: nested side branch");
    if (!side_st) HIPCHECK(hipStreamCreateWithFlags(&side_st, hipStreamNonBlocking));
    hipEvent_t e = side_event();
    hipStream_t sd = side_st;
    op([e, sd](hipStream_t s) {
      HIPCHECK(hipEventRecord(e, s));
      HIPCHECK(hipStreamWaitEvent(sd, e, 0));
    });
    main_st = st;
    st = sd;   // uploads of the branch go in its order
    op.side = sd;
    side_pending = true;
  }
  void end_side() {
    if (!op.side) return;
    op.side = nullptr;
    st = main_st;
  }
  void join_side() {
    if (!side_pending) return;
    end_side();
    hipEvent_t e = side_event();
    hipStream_t sd = side_st;
    op([e, sd](hipStream_t s) {
      HIPCHECK(hipEventRecord(e, sd));
      HIPCHECK(hipStreamWaitEvent(s, e, 0));
    });
    side_pending = false;
  }

  void set(const std::string& name, double* p, const char* axes, int sym = 0) {
    TensorRef t{p, axes, {}};
    t.sym = sym;
    int r = (int)strlen(axes);
    t.stride.assign(r, 1);
    for (int k = r - 2; k >= 0; --k) t.stride[k] = t.stride[k + 1] * d.len(axes[k + 1]);
    t.lim = t.stride[0] * d.len(axes[0]);
    tensors[name] = t;
  }
  void set_view(const std::string& name, double* p, const char* axes, std::vector<long long> stride,
                long long lim) {
    tensors[name] = TensorRef{p, axes, stride, lim};
  }

  // ---- Coulomb blocks J(X1 X2 | X3 X4)[p][q][r][s] = sum_Q B[Q][p][q] B[Q][r][s] ----
  // (optionally the first index in [off1, off1 + n1) and the third in [off3, off3 + n3) of
  // their spaces)
  void build_j(char s1, char s2, char s3, char s4, int off1, int n1, double* out, int off3 = 0,
               int n3 = -1, int tri = 0) {
    int N = d.nC + d.nA + d.nV;
    GettDesc g;
    g.nm = 2; g.nn = 2; g.nk = 1;
    g.md[0] = n1; g.md[1] = d.len(s2);
    g.nd[0] = n3 < 0 ? d.len(s3) : n3; g.nd[1] = d.len(s4);
    g.kd[0] = M;
    g.M = g.md[0] * g.md[1];
    g.N = g.nd[0] * g.nd[1];
    g.K = M;
    const double* A0 = B + (long long)(d.off(s1) + off1) * N + d.off(s2);
    const double* B0 = B + (long long)(d.off(s3) + off3) * N + d.off(s4);
    g.am[0] = N; g.am[1] = 1; g.ak[0] = (long long)N * N;
    g.bk[0] = (long long)N * N; g.bn[0] = N; g.bn[1] = 1;
    g.cm[0] = (long long)g.md[1] * g.N; g.cm[1] = g.N;
    g.cn[0] = g.nd[1]; g.cn[1] = 1;
    g.alpha = 1.0; g.beta = 0;
    long long nB = (long long)M * N * N;
    check_view("B (first pair)", nB - (A0 - B), {g.am[0], g.am[1], g.ak[0]}, {g.md[0], g.md[1], M});
    check_view("B (second pair)", nB - (B0 - B), {g.bn[0], g.bn[1], g.bk[0]}, {g.nd[0], g.nd[1], M});
    gett_prepare(g);   // may merge components: the checks above use the unmerged ones
    g.tri = tri;
    gett(g, A0, B0, out, kRoleIntegrals);
  }
  double* jblock(const std::string& key) {
    auto it = jblocks.find(key);
    if (it != jblocks.end()) return it->second;
    size_t n = (size_t)d.len(key[0]) * d.len(key[1]) * d.len(key[2]) * d.len(key[3]);
    double* p = pool.alloc(n);
    build_j(key[0], key[1], key[2], key[3], 0, d.len(key[0]), p);
    jblocks[key] = p;
    return p;
  }

  static char promote(char s) { return (s == 'C' || s == 'A' || s == 'H') ? 'H' : 'P'; }

  // Canonical chemist order of a J factor: H before P inside each pair, then pairs HH < HP < PP.
  static void canon_j(const std::string& L, const std::map<char, char>& sp, std::string& letters,
                      std::string& key) {
    std::string l = L;
    auto pr = [&](char c) { return promote(sp.at(c)); };
    if (pr(l[0]) == 'P' && pr(l[1]) == 'H') std::swap(l[0], l[1]);
    if (pr(l[2]) == 'P' && pr(l[3]) == 'H') std::swap(l[2], l[3]);
    auto rank = [&](char a, char b) { return (pr(a) == 'P') + (pr(b) == 'P'); };
    if (rank(l[0], l[1]) > rank(l[2], l[3])) l = l.substr(2, 2) + l.substr(0, 2);
    letters = l;
    key = std::string() + pr(l[0]) + pr(l[1]) + pr(l[2]) + pr(l[3]);
  }

  // ---- letter ranges (with an optional batched letter) ----
  struct LetterRange {
    std::map<char, int> off, len;   // offset inside the letter's own space, length
  };

  Opnd factor_view(const TFactor& f, const std::map<char, char>& sp, const LetterRange& lr,
                   const double* jbatch, char batch_letter) {
    Opnd o;
    if (f.tensor == "J") {
      std::string L, key;
      canon_j(f.letters, sp, L, key);
      const double* base;
      std::vector<int> dims(4);
      std::vector<int> extra(4, 0);
      if (key == "PPPP") {
        base = jbatch;
        if (!jbatch || L[0] != batch_letter) throw Error(DSRG_E_HIP, "internal: unbatched (PP|PP) block");
        dims[0] = lr.len.at(L[0]);
        for (int k = 1; k < 4; ++k) dims[k] = d.len('P');
      } else {
        base = jblock(key);
        for (int k = 0; k < 4; ++k) dims[k] = d.len(key[k]);
      }
      std::vector<long long> stride(4, 1);
      for (int k = 2; k >= 0; --k) stride[k] = stride[k + 1] * dims[k + 1];
      long long off = 0;
      for (int k = 0; k < 4; ++k) {
        char l = L[k];
        int pos = d.off(sp.at(l)) - d.off(key[k]) + lr.off.at(l);
        if (key == "PPPP" && k == 0) pos = 0;   // the batch buffer starts at the batch
        off += pos * stride[k];
      }
      o.p = base + off;
      o.letters = L;
      o.stride = stride;
      o.lim = (long long)dims[0] * stride[0] - off;
      return o;
    }
    std::string name = f.tensor + "." + f.block;
    auto it = tensors.find(name);
    if (it == tensors.end()) throw Error(DSRG_E_HIP, "internal: tensor " + name + " not bound");
    const TensorRef& t = it->second;
    long long off = 0;
    for (size_t k = 0; k < f.letters.size(); ++k) {
      char l = f.letters[k];
      off += (long long)(d.off(sp.at(l)) - d.off(t.axes[k]) + lr.off.at(l)) * t.stride[k];
    }
    o.p = t.p + off;
    o.letters = f.letters;
    o.stride = t.stride;
    o.lim = t.lim - off;
    return o;
  }

  // Descriptor of C[m][n] = sum_k a[m, k] b[k, n] for two operands: the free letters of a
  // (in a's order) form m, those of b form n, the shared letters form k.  C strides are left
  // to the caller, which then runs gett_prepare.
  GettDesc pair_desc(const Opnd& a, const Opnd& b, const LetterRange& lr, std::string& ml,
                     std::string& nl) {
    std::string kl;
    std::vector<long long> am, ak, bk, bn;
    ml.clear();
    nl.clear();
    for (size_t i = 0; i < a.letters.size(); ++i) {
      char l = a.letters[i];
      size_t j = b.letters.find(l);
      if (j == std::string::npos) { ml += l; am.push_back(a.stride[i]); }
      else { kl += l; ak.push_back(a.stride[i]); bk.push_back(b.stride[j]); }
    }
    for (size_t j = 0; j < b.letters.size(); ++j)
      if (a.letters.find(b.letters[j]) == std::string::npos) { nl += b.letters[j]; bn.push_back(b.stride[j]); }
    GettDesc g;
    g.nm = (int)ml.size(); g.nn = (int)nl.size(); g.nk = (int)kl.size();
    if (g.nm > kMaxComp || g.nn > kMaxComp || g.nk > kMaxComp) throw Error(DSRG_E_HIP, "internal: rank");
    long long Mx = 1, Nx = 1, Kx = 1;
    for (int i = 0; i < g.nm; ++i) { g.md[i] = lr.len.at(ml[i]); g.am[i] = am[i]; Mx *= g.md[i]; }
    for (int i = 0; i < g.nn; ++i) { g.nd[i] = lr.len.at(nl[i]); g.bn[i] = bn[i]; Nx *= g.nd[i]; }
    for (int i = 0; i < g.nk; ++i) { g.kd[i] = lr.len.at(kl[i]); g.ak[i] = ak[i]; g.bk[i] = bk[i]; Kx *= g.kd[i]; }
    if (Mx >= (1LL << 31) || Nx >= (1LL << 31) || Kx >= (1LL << 31))
      throw Error(DSRG_E_UNSUPPORTED, "contraction dimension exceeds 2^31");
    g.M = (int)Mx; g.N = (int)Nx; g.K = (int)Kx;
    check_operand("contraction A", a, lr);
    check_operand("contraction B", b, lr);
    return g;
  }

  // Contiguous result operand with letters ml + nl, laid out row-major in the order of
  // `layout` (default: ml + nl); sets the C strides of g.
  Opnd result_operand(GettDesc& g, const std::string& ml, const std::string& nl, const LetterRange& lr,
                      const std::string& layout = "") {
    Opnd r;
    r.letters = ml + nl;
    r.lim = (long long)g.M * g.N;
    const std::string lay = layout.empty() ? r.letters : layout;
    if (lay.size() != r.letters.size()) throw Error(DSRG_E_HIP, "internal: result layout");
    r.stride.assign(r.letters.size(), 1);
    long long st = 1;
    for (int k = (int)lay.size() - 1; k >= 0; --k) {
      size_t pos = r.letters.find(lay[k]);
      if (pos == std::string::npos) throw Error(DSRG_E_HIP, "internal: result layout letter");
      r.stride[pos] = st;
      st *= lr.len.at(lay[k]);
    }
    for (int i = 0; i < g.nm; ++i) g.cm[i] = r.stride[i];
    for (int i = 0; i < g.nn; ++i) g.cn[i] = r.stride[g.nm + i];
    g.alpha = 1.0;
    g.beta = 0;
    gett_prepare(g);   // after the C strides: it merges free components of A/B and C
    {
      std::vector<long long> cs;
      std::vector<int> len;
      for (int i = 0; i < g.nm; ++i) { cs.push_back(g.cm[i]); len.push_back(g.md[i]); }
      for (int i = 0; i < g.nn; ++i) { cs.push_back(g.cn[i]); len.push_back(g.nd[i]); }
      check_view("contraction result", r.lim, cs, len);
    }
    return r;
  }

  // contract two operands into a new contiguous temporary
  Opnd contract(const Opnd& a, const Opnd& b, const LetterRange& lr, std::vector<double*>& temps) {
    std::string ml, nl;
    GettDesc g = pair_desc(a, b, lr, ml, nl);
    Opnd r = result_operand(g, ml, nl, lr);
    double* out = pool_temp((size_t)r.lim, temps);
    r.p = out;
    gett(g, a.p, b.p, out, role_now);
    return r;
  }

  // Greedy pairwise order: the pair whose combined letters span the fewest elements.
  static std::pair<size_t, size_t> pick_pair(const std::vector<Opnd>& ops, const LetterRange& lr) {
    size_t bi = 0, bj = 1;
    double best = 1e300;
    for (size_t i = 0; i < ops.size(); ++i)
      for (size_t j = i + 1; j < ops.size(); ++j) {
        std::string u = ops[i].letters;
        for (char c : ops[j].letters)
          if (u.find(c) == std::string::npos) u += c;
        double c = 1;
        for (char l : u) c *= lr.len.at(l);
        if (c < best) { best = c; bi = i; bj = j; }
      }
    return {bi, bj};
  }

  void check_operand(const char* what, const Opnd& o, const LetterRange& lr) {
    std::vector<int> len;
    for (char c : o.letters) len.push_back(lr.len.at(c));
    check_view(what, o.lim, o.stride, len);
  }


  // temporaries: grow-only arena reused across products (single stream, so reuse is
  // ordered after every earlier use)
  std::vector<std::pair<double*, size_t>> free_tmp;
  double* pool_temp(size_t n, std::vector<double*>& temps) {
    size_t best = free_tmp.size();
    for (size_t i = 0; i < free_tmp.size(); ++i)
      if (free_tmp[i].second >= n && (best == free_tmp.size() || free_tmp[i].second < free_tmp[best].second))
        best = i;
    double* p;
    size_t sz;
    if (best < free_tmp.size()) {
      p = free_tmp[best].first;
      sz = free_tmp[best].second;
      free_tmp.erase(free_tmp.begin() + best);
    } else {
      p = pool.alloc(n);
      sz = n;
    }
    temps.push_back(p);
    tmp_size[p] = sz;
    return p;
  }
  std::map<double*, size_t> tmp_size;
  void release_temps(std::vector<double*>& temps) {
    for (double* t : temps) free_tmp.push_back({t, tmp_size[t]});
    temps.clear();
  }

  // Execute one product; outputs by name ("O1.a" -> TensorRef) or scalar slots.
  void run_product(const TProduct& P, const LetterRange& lr, const double* jbatch, char batch_letter,
                   std::map<std::string, TensorRef>& outs, double* slot, double& slot_coef,
                   double flops_scale_ladder) {
    for (auto& kv : lr.len)
      if (kv.second == 0) return;
    std::vector<Opnd> ops;
    for (auto& f : P.f) ops.push_back(factor_view(f, P.space, lr, jbatch, batch_letter));
    std::vector<double*> temps;
    double f0 = gett_flops;
    // direct path: two factors, one scatter into a tensor output
    if (ops.size() == 2 && P.s.size() == 1 && !P.res.empty()) {
      const TScatter& s = P.s[0];
      const TensorRef& o = outs.at(s.tensor + "." + s.block);
      contract_into(ops[0], ops[1], lr, P.space, s, o);
      if (flops_scale_ladder > 0) ladder_flops += gett_flops - f0;
      return;
    }
    while (ops.size() > 2 || (ops.size() == 2 && !P.res.empty())) {
      auto [bi, bj] = pick_pair(ops, lr);
      Opnd r = contract(ops[bi], ops[bj], lr, temps);
      ops.erase(ops.begin() + bj);
      ops[bi] = r;
    }
    if (P.res.empty()) {
      // final scalar: dot product of the last two operands
      if (ops.size() != 2) throw Error(DSRG_E_HIP, "internal: scalar product shape");
      const Opnd& a = ops[0];
      const Opnd& b = ops[1];
      DotDesc dd;
      dd.nk = (int)a.letters.size();
      dd.K = 1;
      for (int i = 0; i < dd.nk; ++i) {
        char l = a.letters[i];
        size_t j = b.letters.find(l);
        dd.kd[i] = lr.len.at(l);
        dd.as[i] = a.stride[i];
        dd.bs[i] = b.stride[j];
        dd.K *= dd.kd[i];
      }
      check_operand("dot A", a, lr);
      check_operand("dot B", b, lr);
      {
        const double *pa = a.p, *pb = b.p;
        double* part = partial;
        op([dd, pa, pb, part, slot](hipStream_t s) { launch_dot(dd, pa, pb, part, slot, s); });
      }
      n_launch += 2;
      gett_flops += 2.0 * dd.K;
      double c = 0;
      for (auto& s : P.s) c += s.coef;
      slot_coef = c;
    } else {
      const Opnd& r = ops[0];
      for (auto& s : P.s) {
        const TensorRef& o = outs.at(s.tensor + "." + s.block);
        ScatterDesc sd;
        sd.rank = (int)s.letters.size();
        sd.n = 1;
        long long ooff = 0;
        for (int k = 0; k < sd.rank; ++k) {
          char l = s.letters[k];
          sd.d[k] = lr.len.at(l);
          sd.ss[k] = r.stride[r.letters.find(l)];
          sd.so[k] = o.stride[k];
          ooff += (long long)(d.off(P.space.at(l)) - d.off(o.axes[k]) + lr.off.at(l)) * o.stride[k];
          sd.n *= sd.d[k];
        }
        sd.coef = s.coef;
        check_operand("scatter source", r, lr);
        {
          std::vector<long long> so(sd.so, sd.so + sd.rank);
          std::vector<int> len(sd.d, sd.d + sd.rank);
          check_view("scatter target", o.lim - ooff, so, len);
        }
        {
          const double* src = r.p;
          double* dst = o.p + ooff;
          op([sd, src, dst](hipStream_t s) { launch_scatter(sd, src, dst, s); });
        }
        ++n_launch;
      }
    }
    release_temps(temps);
    if (flops_scale_ladder > 0) ladder_flops += gett_flops - f0;
  }

  void contract_into(const Opnd& a, const Opnd& b, const LetterRange& lr,
                     const std::map<char, char>& sp, const TScatter& s, const TensorRef& o) {
    std::string ml, nl, kl;
    GettDesc g;
    long long ooff = 0;
    std::map<char, long long> ostr;
    for (size_t k = 0; k < s.letters.size(); ++k) {
      char l = s.letters[k];
      ostr[l] = o.stride[k];
      ooff += (long long)(d.off(sp.at(l)) - d.off(o.axes[k]) + lr.off.at(l)) * o.stride[k];
    }
    for (size_t i = 0; i < a.letters.size(); ++i) {
      char l = a.letters[i];
      size_t j = b.letters.find(l);
      if (j == std::string::npos) {
        g.md[g.nm] = lr.len.at(l); g.am[g.nm] = a.stride[i]; g.cm[g.nm] = ostr.at(l); ++g.nm;
      } else {
        g.kd[g.nk] = lr.len.at(l); g.ak[g.nk] = a.stride[i]; g.bk[g.nk] = b.stride[j]; ++g.nk;
      }
    }
    for (size_t j = 0; j < b.letters.size(); ++j) {
      char l = b.letters[j];
      if (a.letters.find(l) == std::string::npos) {
        g.nd[g.nn] = lr.len.at(l); g.bn[g.nn] = b.stride[j]; g.cn[g.nn] = ostr.at(l); ++g.nn;
      }
    }
    long long Mx = 1, Nx = 1, Kx = 1;
    for (int i = 0; i < g.nm; ++i) Mx *= g.md[i];
    for (int i = 0; i < g.nn; ++i) Nx *= g.nd[i];
    for (int i = 0; i < g.nk; ++i) Kx *= g.kd[i];
    if (Mx >= (1LL << 31) || Nx >= (1LL << 31) || Kx >= (1LL << 31))
      throw Error(DSRG_E_UNSUPPORTED, "contraction dimension exceeds 2^31");
    g.M = (int)Mx; g.N = (int)Nx; g.K = (int)Kx;
    gett_prepare(g);
    g.alpha = s.coef;
    g.beta = 1;
    check_operand("contraction A", a, lr);
    check_operand("contraction B", b, lr);
    {
      std::vector<long long> cs;
      std::vector<int> len;
      for (int i = 0; i < g.nm; ++i) { cs.push_back(g.cm[i]); len.push_back(g.md[i]); }
      for (int i = 0; i < g.nn; ++i) { cs.push_back(g.cn[i]); len.push_back(g.nd[i]); }
      check_view("contraction target", o.lim - ooff, cs, len);
    }
    gett(g, a.p, b.p, o.p + ooff, role_now);
  }

  static bool is_pppp(const TProduct& P, std::string* jl) {
    for (auto& f : P.f)
      if (f.tensor == "J") {
        std::string L, key;
        canon_j(f.letters, P.space, L, key);
        if (key == "PPPP") {
          if (jl) *jl = L;
          return true;
        }
      }
    return false;
  }

  LetterRange full_range(const TProduct& P) const {
    LetterRange lr;
    for (auto& kv : P.space) {
      lr.off[kv.first] = 0;
      lr.len[kv.first] = d.len(kv.second);
    }
    return lr;
  }

  // Host copies behind asynchronous uploads; they live until the call has synchronised.
  std::deque<std::vector<char>> hold;
  template <class T>
  T* upload(const std::vector<T>& v) {
    if (v.empty()) return nullptr;
    size_t bytes = v.size() * sizeof(T);
    double* dp = pool.alloc((bytes + 7) / 8);
    hold.emplace_back((const char*)v.data(), (const char*)v.data() + bytes);
    const char* src = hold.back().data();
    if (op.defer)
      op([dp, src, bytes](hipStream_t s) { HIPCHECK(hipMemcpyAsync(dp, src, bytes, hipMemcpyHostToDevice, s)); });
    else
      HIPCHECK(hipMemcpyAsync(dp, src, bytes, hipMemcpyHostToDevice, st));
    return (T*)dp;
  }

  // A grouped launch, bracketed by events when profiling.
  // A grouped launch.  With profiling, the contraction launches (timed = true) are
  // bracketed by events and counted under the grouped role (items in M, workgroups in N of
  // the profile record); helper launches are not.
  void group_launch(double flops, DevOp launch, bool timed = false, int items = 0, int tiles = 0,
                    double bytes = 0, int role = kRoleGrouped, bool big = false) {
    Rec r{nullptr, nullptr, role, flops, 0, 0, 0, 0, 0, 0, -2};
    r.bytes = bytes;
    r.big = big ? 1 : 0;
    timed = timed && profile;
    r.M = items;
    r.N = tiles;
    r.product = use_id * 10000 + 9000 + group_level++;
    if (timed) {
      HIPCHECK(hipEventCreate(&r.a));
      HIPCHECK(hipEventCreate(&r.b));
      HIPCHECK(hipEventRecord(r.a, st));
    }
    op(std::move(launch));
    if (timed) {
      HIPCHECK(hipEventRecord(r.b, st));
      recs.push_back(r);
    }
    gett_flops += flops;
    ++n_launch;
  }

  // Tile shape of a grouped item: the square 64 x 64 one unless it pads more than 1.8
  // times the work of the thinnest fit (a 16 x 128 or 128 x 16 workgroup step costs about
  // as long as a 64 x 64 one in these latency-bound launches but covers half the
  // outputs); 128 x 128 when it pads at most 10 % more than the chosen small shape (four
  // times the work per loaded element) and the k range is long (short ones ran slower
  // that way).
  // C^T = B^T A^T: the same contraction with the roles of m and n (and of A and B) swapped
  static void transpose_item(GroupItem& it) {
    GettDesc& g = it.g;
    std::swap(g.M, g.N);
    std::swap(g.nm, g.nn);
    for (int c = 0; c < kMaxComp; ++c) {
      std::swap(g.md[c], g.nd[c]);
      std::swap(g.am[c], g.bn[c]);
      std::swap(g.ak[c], g.bk[c]);
      std::swap(g.cm[c], g.cn[c]);
    }
    std::swap(g.a_kfast, g.b_kfast);
    std::swap(it.A, it.B);
  }
  static void group_shape(GroupItem& it) {
    GettDesc& g = it.g;
    if (g.K <= kGettBK && std::min(g.M, g.N) <= kGroupRowN) {
      // one output row per thread along the long free dimension (operands swapped later
      // when that is N)
      it.shape = kGroupRowShape;
      it.tiles_m = (std::max(g.M, g.N) + kGroupRows - 1) / kGroupRows;
      it.tiles_n = 1;
      return;
    }
    long long bestw = -1, w0 = -1;
    int best = 0;
    for (int sh = 0; sh < kGroupShapes; ++sh) {
      if (sh == kGroupBigShape) continue;
      const long long tm = (g.M + kGroupTiles[sh][0] - 1) / kGroupTiles[sh][0];
      const long long tn = (g.N + kGroupTiles[sh][1] - 1) / kGroupTiles[sh][1];
      const long long w = tm * kGroupTiles[sh][0] * tn * kGroupTiles[sh][1];
      if (sh == 0) w0 = w;
      if (bestw < 0 || w < bestw) {
        bestw = w;
        best = sh;
      }
    }
    if (w0 * 5 <= bestw * 9) {
      best = 0;
      bestw = w0;
    }
    it.shape = best;
    it.tiles_m = (g.M + kGroupTiles[best][0] - 1) / kGroupTiles[best][0];
    it.tiles_n = (g.N + kGroupTiles[best][1] - 1) / kGroupTiles[best][1];
    if (g.M >= 128 && g.N >= 128 && g.steps >= 128) {
      const long long tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
      if (tm * tn * 128 * 128 * 10 <= bestw * 11) {
        it.shape = kGroupBigShape;
        it.tiles_m = (int)tm;
        it.tiles_n = (int)tn;
        gett_unpack_k(g);   // the 128 x 128 group tile walks plain k steps
      }
    }
  }

  // The Coulomb blocks (except (PP|PP)) of a call, in one grouped launch when they are all
  // small (each at most 2^22 elements), else one launch each.
  void prebuild_j(const std::vector<std::string>& keys) {
    std::vector<std::string> todo;
    bool small = grouped;
    for (auto& k : keys)
      if (!jblocks.count(k) && std::find(todo.begin(), todo.end(), k) == todo.end()) {
        todo.push_back(k);
        if ((long long)d.len(k[0]) * d.len(k[1]) * d.len(k[2]) * d.len(k[3]) > (1LL << 22)) small = false;
      }
    if (todo.empty()) return;
    if (!small || todo.size() < 2) {
      for (auto& k : todo) jblock(k);
      return;
    }
    const int N = d.nC + d.nA + d.nV;
    const long long nB = (long long)M * N * N;
    std::vector<GroupItem> items;
    std::vector<int> tile_item;
    double fl = 0, bytes = 0;
    int tiles = 0;
    for (auto& k : todo) {
      GettDesc g;
      g.nm = 2; g.nn = 2; g.nk = 1;
      g.md[0] = d.len(k[0]); g.md[1] = d.len(k[1]);
      g.nd[0] = d.len(k[2]); g.nd[1] = d.len(k[3]);
      g.kd[0] = M;
      g.M = g.md[0] * g.md[1];
      g.N = g.nd[0] * g.nd[1];
      g.K = M;
      g.am[0] = N; g.am[1] = 1; g.ak[0] = (long long)N * N;
      g.bk[0] = (long long)N * N; g.bn[0] = N; g.bn[1] = 1;
      g.cm[0] = (long long)g.md[1] * g.N; g.cm[1] = g.N;
      g.cn[0] = g.nd[1]; g.cn[1] = 1;
      g.alpha = 1.0; g.beta = 0;
      const double* A0 = B + (long long)d.off(k[0]) * N + d.off(k[1]);
      const double* B0 = B + (long long)d.off(k[2]) * N + d.off(k[3]);
      check_view("B (first pair)", nB - (A0 - B), {g.am[0], g.am[1], g.ak[0]}, {g.md[0], g.md[1], M});
      check_view("B (second pair)", nB - (B0 - B), {g.bn[0], g.bn[1], g.bk[0]}, {g.nd[0], g.nd[1], M});
      gett_prepare(g);
      double* out = pool.alloc((size_t)g.M * g.N);
      jblocks[k] = out;
      GroupItem it;
      it.g = g;
      it.A = A0;
      it.B = B0;
      it.C = out;
      group_shape(it);
      it.g.kchunk = it.g.steps;
      it.g.part = nullptr;
      it.splits = 1;
      if (it.shape == kGroupRowShape && it.g.N > kGroupRowN) transpose_item(it);
      gett_magic(it.g);
      if (it.shape == kGroupBigShape) {   // not with K = n_aux < 128 k steps; kept general
        for (auto& kk : todo)
          if (kk != k) jblocks.erase(kk);
        jblocks.erase(k);
        for (auto& kk : todo) jblock(kk);
        return;
      }
      it.tile0 = tiles;
      const int t = it.tiles_m * it.tiles_n;
      for (int q = 0; q < t; ++q) tile_item.push_back((int)items.size());
      tiles += t;
      items.push_back(it);
      fl += 2.0 * g.M * (double)g.N * g.K;
      bytes += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N);
    }
    GroupItem* d_items = upload(items);
    int* d_map = upload(tile_item);
    const int n = (int)items.size();
    const int lo = prec;
    group_launch(fl, [d_items, d_map, n, tiles, lo](hipStream_t s) {
      launch_gett_group(d_items, d_map, n, tiles, false, lo, s, true);
    }, true, n, tiles, bytes, kRoleIntegrals);
  }

  // Sub-spaces of an output axis covered by a letter's space: bit 0 is the lower part of
  // the axis (A of P, C of H, all of A), bit 1 the upper part (V of P, A of H).
  static unsigned covers(char axis, char letter_space) {
    if (axis == 'A' && letter_space == 'A') return 1;
    if (axis == 'P') {
      if (letter_space == 'P') return 3;
      if (letter_space == 'A') return 1;
      if (letter_space == 'V') return 2;
    } else if (axis == 'H') {
      if (letter_space == 'H') return 3;
      if (letter_space == 'C') return 1;
      if (letter_space == 'A') return 2;
    }
    throw Error(DSRG_E_HIP, "internal: output axis/letter space pair");
  }

  // Components in the order of a's strides, largest first, so that the index the dot
  // walks fastest is a's contiguous one (ties: b's strides).
  static DotDesc dot_desc(const Opnd& a, const Opnd& b, const LetterRange& lr) {
    DotDesc dd;
    dd.nk = (int)a.letters.size();
    if (dd.nk > 2 * kMaxComp || a.letters.size() != b.letters.size())
      throw Error(DSRG_E_HIP, "internal: scalar product shape");
    std::vector<int> ord(dd.nk);
    for (int i = 0; i < dd.nk; ++i) ord[i] = i;
    auto bstride = [&](int i) {
      const size_t j = b.letters.find(a.letters[i]);
      return j == std::string::npos ? 0LL : std::llabs(b.stride[j]);
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
      const long long sx = std::llabs(a.stride[x]), sy = std::llabs(a.stride[y]);
      return sx != sy ? sx > sy : bstride(x) > bstride(y);
    });
    dd.K = 1;
    for (int oi = 0; oi < dd.nk; ++oi) {
      const int i = ord[oi];
      char l = a.letters[i];
      size_t j = b.letters.find(l);
      if (j == std::string::npos) throw Error(DSRG_E_HIP, "internal: scalar product letters");
      dd.kd[oi] = lr.len.at(l);
      dd.as[oi] = a.stride[i];
      dd.bs[oi] = b.stride[j];
      dd.K *= dd.kd[oi];
    }
    return dd;
  }

  // Grouped execution of the products of one use: every pairwise contraction writes its
  // own temporary, contractions at the same depth of their product's chain run in one
  // launch, scalar products end in one grouped dot launch and tensor products in one
  // gather per output tensor (fixed entry order, so the sums are deterministic).  Returns
  // false, having launched nothing, when the temporaries would exceed group_cap bytes.
  bool run_grouped(const std::vector<std::pair<int, const TProduct*>>& prods,
                   std::map<std::string, TensorRef>& outs, double* scalar_out,
                   const std::function<void()>& on_start = nullptr) {
    struct Fix {
      long long a, b, c;   // arena offsets of A, B, C (-1: not a temporary)
    };
    std::vector<std::vector<GroupItem>> lev;
    std::vector<std::vector<Fix>> levfix;
    std::vector<DotItem> dots;
    std::vector<std::pair<long long, long long>> dfix;
    std::vector<double> dcoef;
    std::vector<int> dslot;   // scalar slot of each dot (scalar_slots), 0 without slots
    struct GEnt {
      GatherEntry e;
      long long sfix;
      unsigned mask;   // classes this entry contributes to
    };
    std::map<std::string, std::vector<GEnt>> gents;
    long long arena = 0;
    auto take = [&](long long n) {
      long long o = arena;
      arena += (n + 31) / 32 * 32;
      return o;
    };
    for (auto& pp : prods) {
      const TProduct& P = *pp.second;
      LetterRange lr = full_range(P);
      bool empty = false;
      for (auto& kv : lr.len)
        if (kv.second == 0) empty = true;
      if (empty) continue;
      std::vector<Opnd> ops;
      for (auto& f : P.f) ops.push_back(factor_view(f, P.space, lr, nullptr, 0));
      size_t level = 0;
      while (ops.size() > 2 || (ops.size() == 2 && !P.res.empty())) {
        auto [bi, bj] = pick_pair(ops, lr);
        std::string ml, nl;
        GettDesc g = pair_desc(ops[bi], ops[bj], lr, ml, nl);
        // the final result of a tensor product is laid out like its first output, so the
        // gather reads that entry with unit stride
        const bool last = ops.size() == 2 && !P.res.empty();
        // the operand a scalar product's final dot pairs with this result, if any: the
        // result takes its memory order so the dot reads both contiguously
        std::string lay = last ? P.s[0].letters : std::string();
        if (P.res.empty() && ops.size() == 3) {
          const Opnd& o = ops[3 - bi - bj];
          std::string mine = ml + nl, other = o.letters;
          std::string s1 = mine, s2 = other;
          std::sort(s1.begin(), s1.end());
          std::sort(s2.begin(), s2.end());
          if (s1 == s2) {
            std::vector<int> ord(other.size());
            for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
              return std::llabs(o.stride[x]) > std::llabs(o.stride[y]);
            });
            for (int i : ord) lay += other[i];
          }
        }
        Opnd r = result_operand(g, ml, nl, lr, lay);
        r.toff = take(r.lim);
        if (lev.size() <= level) {
          lev.resize(level + 1);
          levfix.resize(level + 1);
        }
        GroupItem it;
        it.g = g;
        it.A = ops[bi].p;
        it.B = ops[bj].p;
        lev[level].push_back(it);
        levfix[level].push_back({ops[bi].toff, ops[bj].toff, r.toff});
        ops.erase(ops.begin() + bj);
        ops[bi] = r;
        ++level;
      }
      if (P.res.empty()) {
        if (ops.size() != 2) throw Error(DSRG_E_HIP, "internal: scalar product shape");
        check_operand("dot A", ops[0], lr);
        check_operand("dot B", ops[1], lr);
        DotItem di;
        di.d = dot_desc(ops[0], ops[1], lr);
        div_magic(di.d.kd, di.d.nk, di.d.dm);
        di.A = ops[0].p;
        di.B = ops[1].p;
        di.nblk = (int)std::max<long long>(1, std::min<long long>(64, (di.d.K + 4095) / 4096));
        dots.push_back(di);
        dfix.push_back({ops[0].toff, ops[1].toff});
        double c = 0;
        for (auto& sc : P.s) c += sc.coef;
        dcoef.push_back(c);
        dslot.push_back(scalar_slots.empty() ? 0 : scalar_slot(P));
      } else {
        const Opnd& r = ops[0];
        check_operand("gather source", r, lr);
        for (auto& sc : P.s) {
          std::string name = sc.tensor + "." + sc.block;
          const TensorRef& o = outs.at(name);
          const int rank = (int)sc.letters.size();
          if (rank > 4 || rank != (int)o.axes.size()) throw Error(DSRG_E_HIP, "internal: gather rank");
          GEnt ge;
          ge.e.src = r.p;
          ge.sfix = r.toff;
          ge.e.coef = sc.coef;
          unsigned allowed[4] = {1, 1, 1, 1};
          long long base = 0;
          for (int k = 0; k < rank; ++k) {
            char l = sc.letters[k];
            size_t pos = r.letters.find(l);
            if (pos == std::string::npos) throw Error(DSRG_E_HIP, "internal: gather letter");
            char ls = P.space.at(l);
            ge.e.ss[k] = r.stride[pos];
            base -= (long long)(d.off(ls) - d.off(o.axes[k])) * r.stride[pos];
            allowed[k] = covers(o.axes[k], ls);
          }
          ge.e.base = base;
          ge.mask = 0;
          for (int c = 0; c < (1 << rank); ++c) {
            bool ok = true;
            for (int k = 0; k < rank; ++k) ok = ok && ((allowed[k] >> ((c >> k) & 1)) & 1);
            if (ok) ge.mask |= 1u << c;
          }
          gents[name].push_back(ge);
        }
      }
    }

    // split-K: a tile's k steps run one after another at about the same time per step
    // whether it has the CU to itself (load latency) or shares it (MFMA), so a level ends no
    // sooner than its longest chain of steps.  Chains are cut to half the level's work per
    // workgroup slot (64 x 64 step units, four such workgroups per CU; at least 8 steps);
    // should the partial tiles not fit beside the temporaries, only items with few tiles and
    // a chain over twice the work per slot are split.  Budget check.
    for (auto& lv : lev)
      for (auto& it : lv) group_shape(it);
    long long part_elems = 0;
    std::vector<std::vector<long long>> poff(lev.size());
    auto plan_splits = [&](bool fine) {
      part_elems = 0;
      for (size_t L = 0; L < lev.size(); ++L) {
        poff[L].clear();
        auto weight = [](const GroupItem& it) {
          return it.shape == kGroupBigShape ? 4LL : 1LL;
        };
        double level_steps = 0;
        for (auto& it : lev[L])
          level_steps += (double)it.tiles_m * it.tiles_n * it.g.steps * weight(it);
        const long long target = std::max<long long>(16, (long long)(level_steps / (4.0 * 256)));
        const long long cap = std::max<long long>(8, target / 2);
        for (auto& it : lev[L]) {
          GettDesc& g = it.g;
          const long long tiles = (long long)it.tiles_m * it.tiles_n, w = weight(it);
          int ns = 1;
          g.kchunk = g.steps;
          if (it.shape == kGroupRowShape) {
            // one pass over k per row, never split
          } else if (fine && g.steps * w > cap + cap / 2) {
            const long long cw = std::max<long long>(1, cap / w);
            const long long want = std::min<long long>((g.steps + cw - 1) / cw, 64);
            const long long chunk = (g.steps + want - 1) / want;
            ns = (int)((g.steps + chunk - 1) / chunk);
            g.kchunk = chunk;
          } else if (!fine && g.steps >= 64 && g.steps > 2 * target && tiles < 64) {
            const long long want = std::min<long long>((g.steps + target - 1) / target,
                                                       std::max<long long>(1, 256 / tiles));
            const long long chunk = (g.steps + want - 1) / want;
            ns = (int)((g.steps + chunk - 1) / chunk);
            g.kchunk = chunk;
          }
          it.splits = ns;
          poff[L].push_back(ns > 1 ? part_elems : -1);
          if (ns > 1) part_elems += (long long)ns * g.M * g.N;
        }
      }
    };
    plan_splits(true);
    if (8 * (arena + part_elems) > group_cap) plan_splits(false);
    long long bytes = 8 * (arena + part_elems);
    if (bytes > group_cap) return false;
    if (on_start) on_start();   // e.g. a side branch that overlaps the launches below

    double* tbase = arena > 0 ? pool.alloc((size_t)arena) : nullptr;
    double* pbase = part_elems > 0 ? pool.alloc((size_t)part_elems) : nullptr;
    auto at = [&](long long off, const double* p) -> const double* { return off >= 0 ? tbase + off : p; };

    // flatten the levels (longest tiles first inside a level) and patch the addresses
    std::vector<GroupItem> items;
    std::vector<ReduceBlock> rblocks;
    struct LevelRange {
      int i0, n, tiles, s0, ns;
      long long red;
      double flops;
      bool big;
      double bytes;
    };
    std::vector<LevelRange> ranges;
    for (size_t L = 0; L < lev.size(); ++L)
     for (int big = 1; big >= 0; --big) {
      std::vector<int> order;
      for (size_t i = 0; i < lev[L].size(); ++i)
        if ((lev[L][i].shape == kGroupBigShape) == (big == 1)) order.push_back((int)i);
      if (order.empty()) continue;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return lev[L][x].g.kchunk > lev[L][y].g.kchunk;
      });
      LevelRange R{(int)items.size(), (int)order.size(), 0, (int)rblocks.size(), 0, 0, 0.0, big == 1, 0.0};
      for (int oi : order) {
        GroupItem it = lev[L][oi];
        const Fix& fx = levfix[L][oi];
        it.A = at(fx.a, it.A);
        it.B = at(fx.b, it.B);
        it.C = tbase + fx.c;
        it.g.part = it.splits > 1 ? pbase + poff[L][oi] : nullptr;
        if (it.shape == kGroupRowShape && it.g.N > kGroupRowN) transpose_item(it);
        gett_magic(it.g);
        it.tile0 = R.tiles;
        long long t = (long long)it.tiles_m * it.tiles_n * it.splits;
        if (R.tiles + t >= (1LL << 31)) throw Error(DSRG_E_UNSUPPORTED, "grouped launch too large");
        R.tiles += (int)t;
        if (it.splits > 1) {
          const long long mn = (long long)it.g.M * it.g.N;
          if (mn >= (1LL << 31)) throw Error(DSRG_E_UNSUPPORTED, "split-K tile too large");
          for (long long e0 = 0; e0 < mn; e0 += 256) {
            rblocks.push_back({(int)items.size() - R.i0, (int)e0});
            ++R.ns;
          }
          R.red += mn;
        }
        R.flops += 2.0 * it.g.M * (double)it.g.N * it.g.K;
        R.bytes += 8.0 * ((double)it.g.M * it.g.K + (double)it.g.K * it.g.N + (double)it.g.M * it.g.N);
        items.push_back(it);
      }
      ranges.push_back(R);
     }
    if (const char* path = getenv("DSRG_GROUP_DUMP")) {
      // planning record for tuning: use, level, M, N, K, splits, k chunk, shape, inner k,
      // steps per inner range, steps
      if (FILE* f = fopen(path, "a")) {
        for (size_t L = 0; L < ranges.size(); ++L)
          for (int i = 0; i < ranges[L].n; ++i) {
            const GroupItem& it = items[ranges[L].i0 + i];
            fprintf(f, "%d,%d,%d,%d,%d,%d,%lld,%d,%d,%d,%lld\n", use_id, (int)L, it.g.M, it.g.N, it.g.K,
                    it.splits, it.g.kchunk, it.shape, it.g.kd[it.g.nk - 1], it.g.ksteps, it.g.steps);
          }
        fclose(f);
      }
    }
    // tile -> item map of every launch (one load per workgroup instead of a search)
    std::vector<int> tile_item;
    std::vector<long long> map0;
    for (auto& R : ranges) {
      map0.push_back((long long)tile_item.size());
      for (int i = 0; i < R.n; ++i) {
        const GroupItem& it = items[R.i0 + i];
        const int t = it.tiles_m * it.tiles_n * it.splits;
        for (int k = 0; k < t; ++k) tile_item.push_back(i);
      }
    }
    GroupItem* d_items = upload(items);
    ReduceBlock* d_rblk = upload(rblocks);
    int* d_map = upload(tile_item);
    for (size_t ri = 0; ri < ranges.size(); ++ri) {
      const LevelRange& R = ranges[ri];
      const GroupItem* it = d_items + R.i0;
      const ReduceBlock* rb = d_rblk + R.s0;
      const int* tm = d_map + map0[ri];
      const int lo = prec;
      group_launch(R.flops, [it, tm, R, lo](hipStream_t s) {
        launch_gett_group(it, tm, R.n, R.tiles, R.big, lo, s);
      }, true, R.n, R.tiles, R.bytes, kRoleGrouped, R.big);
      if (R.ns > 0)
        group_launch(0.0, [it, rb, R](hipStream_t s) { launch_group_reduce(it, rb, R.ns, s); });
    }

    if (scalar_out) {
      // one weighted sum per scalar slot over all dot partials (other slots' weights 0)
      const std::vector<double*> outs_s = scalar_slots.empty() ? std::vector<double*>{scalar_out} : scalar_slots;
      int blocks = 0;
      std::vector<std::vector<double>> bcoef(outs_s.size());
      for (size_t i = 0; i < dots.size(); ++i) {
        dots[i].A = at(dfix[i].first, dots[i].A);
        dots[i].B = at(dfix[i].second, dots[i].B);
        dots[i].blk0 = blocks;
        blocks += dots[i].nblk;
        for (size_t k = 0; k < outs_s.size(); ++k)
          for (int b = 0; b < dots[i].nblk; ++b) bcoef[k].push_back(dslot[i] == (int)k ? dcoef[i] : 0.0);
      }
      if (blocks == 0) {
        for (double* so : outs_s) {
          op([so](hipStream_t s) { launch_fill(so, 1, 0.0, s); });
          ++n_launch;
        }
      } else {
        double* part = pool.alloc((size_t)blocks);
        DotItem* d_dots = upload(dots);
        double fl = 0;
        for (auto& di : dots) fl += 2.0 * di.d.K;
        const int nd = (int)dots.size();
        group_launch(fl, [d_dots, nd, blocks, part](hipStream_t s) {
          launch_dot_group(d_dots, nd, blocks, part, s);
        });
        // every slot's weighted sum in one launch (workgroup k sums slot k in a fixed order)
        for (size_t k0 = 0; k0 < outs_s.size(); k0 += 8) {
          const size_t k1 = std::min(outs_s.size(), k0 + 8);
          std::vector<double> coefs;
          SumOuts so;
          for (size_t k = k0; k < k1; ++k) {
            coefs.insert(coefs.end(), bcoef[k].begin(), bcoef[k].end());
            so.o[so.n++] = outs_s[k];
          }
          double* d_coef = upload(coefs);
          op([blocks, part, d_coef, so](hipStream_t s) { launch_weighted_sums(blocks, part, d_coef, so, s); });
          ++n_launch;
        }
      }
    } else if (!dots.empty()) {
      throw Error(DSRG_E_HIP, "internal: scalar products in a tensor use");
    }

    // every output's gather in one launch (outputs are distinct arrays)
    std::vector<GatherDesc> gds;
    std::vector<std::vector<GatherEntry>> gent;
    long long gblocks = 0;
    for (auto& kv : gents) {
      const TensorRef& o = outs.at(kv.first);
      GatherDesc gd;
      gd.rank = (int)o.axes.size();
      if (gd.rank > 4 || o.lim >= (1LL << 38))
        throw Error(DSRG_E_UNSUPPORTED, "gathered output too large");
      std::vector<GatherEntry> ent;
      for (int k = 0; k < gd.rank; ++k) {
        gd.dim[k] = d.len(o.axes[k]);
        gd.split[k] = o.axes[k] == 'P' ? d.nA : o.axes[k] == 'H' ? d.nC : gd.dim[k];
        if (o.stride[k] != (k + 1 < gd.rank ? o.stride[k + 1] * d.len(o.axes[k + 1]) : 1))
          throw Error(DSRG_E_HIP, "internal: gather output must be contiguous");
      }
      for (int c = 0; c < (1 << gd.rank); ++c) {
        gd.cls[c] = (int)ent.size();
        for (auto& ge : kv.second)
          if ((ge.mask >> c) & 1) {
            GatherEntry e = ge.e;
            e.src = at(ge.sfix, e.src);
            ent.push_back(e);
          }
      }
      gd.cls[1 << gd.rank] = (int)ent.size();
      gd.out = o.p;
      const long long nb = gather_prepare(gd);
      if (nb <= 0) continue;
      if (const char* path = getenv("DSRG_GROUP_DUMP")) {
        // gather record: G, use, output, rank, tpe, workgroups, then per class: entries,
        // elements, entries whose last index has unit stride
        if (FILE* f = fopen(path, "a")) {
          fprintf(f, "G,%d,%s,%d,%d,%lld", use_id, kv.first.c_str(), gd.rank, gd.tpe, nb);
          for (int c = 0; c < (1 << gd.rank); ++c) {
            long long cnt = 1;
            for (int k = 0; k < gd.rank; ++k)
              cnt *= ((c >> k) & 1) ? gd.dim[k] - gd.split[k] : gd.split[k];
            int unit = 0;
            for (int i = gd.cls[c]; i < gd.cls[c + 1]; ++i) unit += ent[i].ss[gd.rank - 1] == 1;
            fprintf(f, ",%d,%lld,%d", gd.cls[c + 1] - gd.cls[c], cnt, unit);
          }
          fprintf(f, "\n");
          fclose(f);
        }
      }
      gd.blk0 = (int)gblocks;
      gblocks += nb;
      if (gblocks >= (1LL << 31)) throw Error(DSRG_E_UNSUPPORTED, "gather launch too large");
      gds.push_back(gd);
      gent.push_back(std::move(ent));
    }
    if (!gds.empty()) {
      for (size_t i = 0; i < gds.size(); ++i) gds[i].ent = upload(gent[i]);
      GatherDesc* d_gd = upload(gds);
      const int ng = (int)gds.size();
      const long long nbk = gblocks;
      join_side();   // a side branch adds into the same outputs: it ends first
      // sources are temporaries of the arena; outputs are contiguous arrays
      bool k32 = arena < (1LL << 31);
      for (auto& kv : gents) k32 = k32 && outs.at(kv.first).lim < (1LL << 31);
      op([d_gd, ng, nbk, k32](hipStream_t s) { launch_gather_multi(d_gd, ng, nbk, s, k32); });
      ++n_launch;
    }
    return true;
  }

  // Products that a use too large to group as a whole still groups: temporaries of the
  // whole chain and the largest contraction below these bounds.
  static constexpr double kSmallProductBytes = 64.0 * (1 << 20), kSmallProductFlops = 2e10;
  // Elements of the temporaries of a product's contraction chain and its largest
  // contraction's flops (the same greedy order as the executors).
  void product_cost(const TProduct& P, double& temp, double& flops) {
    temp = 0;
    flops = 0;
    LetterRange lr = full_range(P);
    for (auto& kv : lr.len)
      if (kv.second == 0) return;
    std::vector<Opnd> ops;
    for (auto& f : P.f) ops.push_back(factor_view(f, P.space, lr, nullptr, 0));
    while (ops.size() > 2 || (ops.size() == 2 && !P.res.empty())) {
      auto [bi, bj] = pick_pair(ops, lr);
      std::string u = ops[bi].letters;
      for (char c : ops[bj].letters)
        if (u.find(c) == std::string::npos) u += c;
      double all = 1, res = 1;
      std::string rl;
      for (char c : u) {
        all *= lr.len.at(c);
        const bool shared = ops[bi].letters.find(c) != std::string::npos &&
                            ops[bj].letters.find(c) != std::string::npos;
        if (!shared) {
          res *= lr.len.at(c);
          rl += c;
        }
      }
      temp += res;
      flops = std::max(flops, 2.0 * all);
      Opnd r;
      r.letters = rl;
      ops.erase(ops.begin() + bj);
      ops[bi] = r;
    }
  }

  // One launch per contraction, temporaries reused from a free list.
  void run_serial(const std::vector<std::pair<int, const TProduct*>>& prods,
                  std::map<std::string, TensorRef>& outs, double* scalar_out) {
    std::vector<double> coefs;
    double* vals = scalar_out ? pool.alloc(prods.size() + 1) : nullptr;
    if (vals) {
      const long long nv = (long long)prods.size() + 1;
      op([vals, nv](hipStream_t s) { launch_fill(vals, nv, 0.0, s); });
    }
    int slot = 0;
    for (auto& pp : prods) {
      cur_product = use_id * 10000 + pp.first;
      const TProduct& P = *pp.second;
      double c = 0;
      run_product(P, full_range(P), nullptr, 0, outs, vals ? vals + slot : nullptr, c, 0);
      if (P.res.empty()) {
        coefs.push_back(c);
        ++slot;
      }
    }
    if (scalar_out) {
      if (coefs.empty()) {
        op([scalar_out](hipStream_t s) { launch_fill(scalar_out, 1, 0.0, s); });
      } else {
        double* coefd = upload(coefs);
        const int nc = (int)coefs.size();
        op([nc, vals, coefd, scalar_out](hipStream_t s) { launch_weighted_sum(nc, vals, coefd, scalar_out, s); });
      }
      ++n_launch;
    }
  }

  // Ladder products O[o] += coef (R0 R1|R2 R3) T[t] that run on unique index pairs, R the
  // block letters with the batch letter R0 first, R0 and R2 free, R1 and R3 summed, every
  // block letter over the whole particle space, both hole letters over the whole hole space.
  // With X[p,q,I,J] = sum_{x,y} (px|qy) T[x,y,I,J] for the real, pair-symmetric integrals:
  //  1: T a same-spin doubles tensor, antisymmetric in its particle pair and in its hole pair:
  //     X is antisymmetric in (p,q) and in (I,J), and the product is c X[o], the sign c
  //     collecting the letter orders;
  //  2: T the opposite-spin doubles, T[x,y,I,J] = T[y,x,J,I], in the order T[R1,R3,h,h'] and
  //     O[R0,R2,h,h']: the product is coef X, whose parts of even and odd particle-pair
  //     symmetry are also of even and odd hole-pair symmetry.
  // 0: any other product.
  bool unique_ladder = true;
  struct LadderTarget {
    double* O;
    double c;
  };
  int pair_ladder(const TProduct& P, char bl, const std::map<std::string, TensorRef>& outs,
                  const double*& Tp, std::vector<LadderTarget>& tg) const {
    tg.clear();
    if (!unique_ladder || P.f.size() != 2 || P.s.empty()) return 0;
    const TFactor* J = nullptr;
    const TFactor* T = nullptr;
    for (auto& f : P.f) {
      if (f.tensor == "J") J = &f;
      else T = &f;
    }
    if (!J || !T || T->tensor != "T2") return 0;
    const int kind = (T->block == "aa" || T->block == "bb") ? 1 : T->block == "ab" ? 2 : 0;
    if (!kind) return 0;
    for (char l : J->letters)
      if (P.space.at(l) != 'P') return 0;
    const std::string R = rotate_first(J->letters, bl, P.space);
    const std::string& t = T->letters;
    auto has = [](const std::string& str, char l) { return str.find(l) != std::string::npos; };
    if (R[0] != bl || !has(P.res, R[0]) || !has(P.res, R[2]) || has(P.res, R[1]) || has(P.res, R[3]))
      return 0;
    if (t.size() != 4) return 0;
    if (P.space.at(t[2]) != 'H' || P.space.at(t[3]) != 'H') return 0;
    if (kind == 1 && !((t[0] == R[1] && t[1] == R[3]) || (t[0] == R[3] && t[1] == R[1]))) return 0;
    if (kind == 2 && (t[0] != R[1] || t[1] != R[3])) return 0;
    auto ti = tensors.find(T->tensor + "." + T->block);
    if (ti == tensors.end() || ti->second.sym != kind) return 0;
    const long long nP = d.len('P'), nH = d.len('H');
    const std::vector<long long> dense{nP * nH * nH, nH * nH, nH, 1};
    auto dense_ok = [&](const TensorRef& r) {
      return r.axes == "PPHH" && r.stride == dense && r.lim >= nP * nP * nH * nH;
    };
    if (!dense_ok(ti->second)) return 0;
    for (const TScatter& S : P.s) {
      const std::string& o = S.letters;
      if (o.size() != 4) return 0;
      if (kind == 1) {
        if (!((o[0] == R[0] && o[1] == R[2]) || (o[0] == R[2] && o[1] == R[0]))) return 0;
        if (!((o[2] == t[2] && o[3] == t[3]) || (o[2] == t[3] && o[3] == t[2]))) return 0;
      } else if (o[0] != R[0] || o[1] != R[2] || o[2] != t[2] || o[3] != t[3]) {
        return 0;
      }
      auto oi = outs.find(S.tensor + "." + S.block);
      if (oi == outs.end() || !dense_ok(oi->second)) return 0;
      double c = S.coef;
      if (kind == 1) c *= (t[0] == R[1] ? 1 : -1) * (o[0] == R[0] ? 1 : -1) * (o[2] == t[2] ? 1 : -1);
      tg.push_back({oi->second.p, c});
    }
    Tp = ti->second.p;
    return kind;
  }

  // Signature of the value of a product: its factors' data (a bound tensor view, or the
  // Coulomb integrals) with letters in a canonical order under the factor's symmetries, the
  // letters' spaces and the result's letter order.  The product is sign times the value of
  // the canonical form.  Products of one signature compute the same result, so one
  // contraction serves all of their scatters.  Empty: no signature (unbound factor).
  bool merge_products = true;
  std::string product_signature(const TProduct& P, int& sign) const {
    sign = 1;
    std::vector<std::string> fs;
    for (auto& f : P.f) {
      std::string L = f.letters;
      std::string key;
      if (f.tensor == "J") {
        // (ab|cd) = (ba|cd) = (ab|dc) = (cd|ab) for real orbitals
        if (L.size() != 4) return "";
        std::string a = L.substr(0, 2), b = L.substr(2, 2);
        if (a[1] < a[0]) std::swap(a[0], a[1]);
        if (b[1] < b[0]) std::swap(b[0], b[1]);
        if (b < a) std::swap(a, b);
        key = "J:" + a + b;
      } else {
        auto it = tensors.find(f.tensor + "." + f.block);
        if (it == tensors.end()) return "";
        const TensorRef& t = it->second;
        if (t.sym && L.size() == 4) {
          // sym 2: T[x][y][i][j] = T[y][x][j][i]; sym 1: antisymmetric in each pair
          const std::string forms[4] = {L, std::string{L[1], L[0], L[2], L[3]},
                                        std::string{L[0], L[1], L[3], L[2]},
                                        std::string{L[1], L[0], L[3], L[2]}};
          const int signs[4] = {1, -1, -1, 1};
          std::string best = L;
          int bs = 1;
          for (int k = 1; k < 4; ++k) {
            if (t.sym == 2 && k != 3) continue;
            if (forms[k] < best) {
              best = forms[k];
              bs = t.sym == 1 ? signs[k] : 1;
            }
          }
          L = best;
          sign *= bs;
        }
        char buf[48];
        snprintf(buf, sizeof(buf), "%p:", (const void*)t.p);
        key = std::string(buf) + t.axes;
        for (long long x : t.stride) key += ":" + std::to_string(x);
        key += ":" + L;
      }
      fs.push_back(key);
    }
    std::sort(fs.begin(), fs.end());
    std::string sig;
    for (auto& x : fs) sig += x + "|";
    for (auto& kv : P.space) {
      sig += kv.first;
      sig += kv.second;
    }
    return sig + "|" + P.res;
  }
  // The products of a use with those of equal signature merged into the first of them.
  Use merged_use(const Use& U) const {
    Use out;
    std::map<std::string, std::pair<size_t, int>> seen;
    for (auto& P : U) {
      int sign = 1;
      std::string sig = merge_products ? product_signature(P, sign) : std::string();
      auto it = sig.empty() ? seen.end() : seen.find(sig);
      if (it == seen.end()) {
        if (!sig.empty()) seen[sig] = {out.size(), sign};
        out.push_back(P);
        continue;
      }
      TProduct& Q = out[it->second.first];
      const double rel = (double)(sign * it->second.second);
      for (TScatter sc : P.s) {
        sc.coef *= rel;
        Q.s.push_back(sc);
      }
    }
    return out;
  }

  // Several scalar uses in one grouped run: each product's scalar scatter names its slot
  // in its block ("0", "1", ...), scalar_slots holds the outputs.  Empty: one scalar.
  std::vector<double*> scalar_slots;
  static int scalar_slot(const TProduct& P) {
    return (P.s.empty() || P.s[0].block.empty()) ? 0 : std::atoi(P.s[0].block.c_str());
  }
  // Run a use of the table into tensor outputs, or (scalar uses) into *scalar_out.
  int use_id = 0;
  int prec = 0;   // DSRG_PRECISION_* of every contraction's products
  int group_level = 0;
  int grouped_uses = 0;
  bool grouped = true;
  long long group_cap = 0;   // bytes of temporaries one grouped use may hold
  // Scatters of a product into a [P][P][H][H] output that form the four images of the
  // pair antisymmetriser, X[pq ij] c, X[qp ij] -c, X[pq ji] -c, X[qp ji] c, become one
  // scatter c X~[pq ij] into a zeroed pre-image X~ of the output, and X += A(X~) once at
  // the end of the use (A: the same four images): a quarter of the scatter (gather)
  // traffic of those products.
  bool collapse_images = true;
  struct PreparedUse {
    Use U;
    std::map<std::string, TensorRef> outs;   // the use's outputs plus its pre-images
    std::vector<std::string> pre;            // names of the pre-images
  };
  // products merged, antisymmetriser images collapsed (pre-images allocated and zeroed)
  PreparedUse prepare_use(const Use& U0, const std::map<std::string, TensorRef>& outs0, bool scalar) {
    PreparedUse pu;
    pu.U = merged_use(U0);
    pu.outs = outs0;
    Use& U = pu.U;
    std::map<std::string, TensorRef>& outs = pu.outs;
    std::vector<std::string>& pre_names = pu.pre;
    if (collapse_images && !scalar) {
      const long long nP = d.len('P'), nH = d.len('H');
      const std::vector<long long> dense{nP * nH * nH, nH * nH, nH, 1};
      auto swap01 = [](std::string o) { std::swap(o[0], o[1]); return o; };
      auto swap23 = [](std::string o) { std::swap(o[2], o[3]); return o; };
      for (auto& P : U) {
        std::vector<TScatter> kept;
        std::vector<bool> used(P.s.size(), false);
        for (size_t a = 0; a < P.s.size(); ++a) {
          if (used[a]) continue;
          const TScatter& S = P.s[a];
          const std::string name = S.tensor + "." + S.block;
          auto oi = outs0.find(name);
          bool quad = false;
          size_t idx[3] = {0, 0, 0};
          if (oi != outs0.end() && S.letters.size() == 4 && oi->second.axes == "PPHH" &&
              oi->second.stride == dense && S.letters[0] != S.letters[1] && S.letters[2] != S.letters[3]) {
            const std::string img[3] = {swap01(S.letters), swap23(S.letters), swap23(swap01(S.letters))};
            const double sg[3] = {-1.0, -1.0, 1.0};
            quad = true;
            for (int k = 0; k < 3 && quad; ++k) {
              bool found = false;
              for (size_t b = 0; b < P.s.size() && !found; ++b)
                if (!used[b] && b != a && P.s[b].tensor == S.tensor && P.s[b].block == S.block &&
                    P.s[b].letters == img[k] && P.s[b].coef == sg[k] * S.coef) {
                  found = true;
                  idx[k] = b;
                }
              quad = found;
            }
          }
          if (!quad) {
            kept.push_back(S);
            used[a] = true;
            continue;
          }
          used[a] = true;
          for (int k = 0; k < 3; ++k) used[idx[k]] = true;
          TScatter R = S;
          R.block += "~";
          kept.push_back(R);
          const std::string pn = S.tensor + "." + R.block;
          if (!outs.count(pn)) {
            outs[pn] = oi->second;   // storage assigned below
            pre_names.push_back(pn);
          }
        }
        P.s = kept;
      }
      // the pre-images of the use in one zeroed block
      long long total = 0;
      for (auto& pn : pre_names) total += outs[pn].lim;
      if (total > 0) {
        double* blk = pool.alloc((size_t)total);
        long long at = 0;
        for (auto& pn : pre_names) {
          outs[pn].p = blk + at;
          at += outs[pn].lim;
        }
        op([blk, total](hipStream_t s) { launch_fill(blk, total, 0.0, s); });
        ++n_launch;
      }
    }
    return pu;
  }
  // the pre-images added into their outputs through the pair antisymmetriser
  // adds the use's pre-images into their outputs, in launches of up to kAntisymList pairs
  void finish_use(const PreparedUse& pu, const std::map<std::string, TensorRef>& outs0) {
    const int nPl = d.len('P'), nHl = d.len('H');
    AntisymList l;
    auto flush = [&] {
      if (l.n == 0) return;
      const AntisymList lc = l;
      op([lc, nPl, nHl](hipStream_t s) { launch_antisym_add_list(lc, nPl, nHl, s); });
      ++n_launch;
      l = AntisymList();
    };
    for (auto& pn : pu.pre) {
      l.X[l.n] = pu.outs.at(pn).p;
      l.O[l.n] = outs0.at(pn.substr(0, pn.size() - 1)).p;
      if (++l.n == kAntisymList) flush();
    }
    flush();
  }
  void run_use(const Use& U0, std::map<std::string, TensorRef>& outs0, double* scalar_out) {
    PreparedUse pu = prepare_use(U0, outs0, scalar_out != nullptr);
    run_use_body(pu.U, pu.outs, scalar_out);
    finish_use(pu, outs0);
  }

  // Several uses whose products are independent in one grouped run of their plain
  // products (their contractions of equal depth share launches); each use's (PP|PP)
  // products and pre-images follow.  scalars[k] is the output of a scalar use (its outs
  // empty).  False, with nothing run but pre-image fills, when the temporaries do not fit
  // the grouping budget together.
  bool run_fused(const std::vector<const Use*>& uses, const std::vector<std::map<std::string, TensorRef>*>& outs,
                 const std::vector<double*>& scalars) {
    if (!grouped || uses.size() != outs.size() || uses.size() != scalars.size()) return false;
    std::vector<PreparedUse> pus;
    for (size_t k = 0; k < uses.size(); ++k) pus.push_back(prepare_use(*uses[k], *outs[k], scalars[k] != nullptr));
    Use all;
    std::vector<Use> pp(uses.size());
    std::map<std::string, TensorRef> all_outs;
    std::vector<double*> slots;
    for (size_t k = 0; k < pus.size(); ++k) {
      const std::string tag = "#" + std::to_string(k);
      int slot = -1;
      if (scalars[k]) {
        slot = (int)slots.size();
        slots.push_back(scalars[k]);
      }
      for (const TProduct& P : pus[k].U) {
        if (is_pppp(P, nullptr)) {
          if (scalars[k]) return false;
          pp[k].push_back(P);
          continue;
        }
        TProduct Q = P;
        for (auto& sc : Q.s) {
          if (Q.res.empty()) {
            if (slot < 0) return false;
            sc.block = std::to_string(slot);
          } else {
            sc.tensor += tag;
          }
        }
        all.push_back(Q);
      }
      for (auto& kv : pus[k].outs) {
        const size_t dot = kv.first.find('.');
        all_outs[kv.first.substr(0, dot) + tag + kv.first.substr(dot)] = kv.second;
      }
    }
    std::vector<std::pair<int, const TProduct*>> plain;
    for (size_t i = 0; i < all.size(); ++i) plain.push_back({(int)i, &all[i]});
    // the (PP|PP) products (own buffers, serial contractions) run on the side stream while
    // the grouped launches run; the gather, which adds into the same outputs, waits for them
    // (not when profiling, whose events time each stream's launches in order)
    bool any_pp = false;
    for (auto& u : pp) any_pp = any_pp || !u.empty();
    const bool overlap = any_pp && !profile && !no_side;
    auto side = [&] {
      fork_side();
      try {
        for (size_t k = 0; k < pus.size(); ++k)
          if (!pp[k].empty()) run_use_body(pp[k], pus[k].outs, nullptr);
      } catch (...) {
        end_side();
        throw;
      }
      end_side();
    };
    scalar_slots = slots;
    const bool ok = run_grouped(plain, all_outs, slots.empty() ? nullptr : slots[0],
                                overlap ? std::function<void()>(side) : nullptr);
    scalar_slots.clear();
    if (!ok) return false;
    join_side();
    ++grouped_uses;
    for (size_t k = 0; k < pus.size(); ++k) {
      if (!overlap && !pp[k].empty()) run_use_body(pp[k], pus[k].outs, nullptr);
      finish_use(pus[k], *outs[k]);
    }
    return true;
  }

  void run_use_body(const Use& U, std::map<std::string, TensorRef>& outs, double* scalar_out) {
    // products with the (PP|PP) block, grouped by the block's letters
    std::map<std::string, std::vector<const TProduct*>> pppp;
    std::vector<std::pair<int, const TProduct*>> plain;
    int pidx = -1;
    for (auto& P : U) {
      ++pidx;
      std::string jl;
      if (is_pppp(P, &jl)) {
        if (scalar_out) throw Error(DSRG_E_HIP, "internal: (PP|PP) block in a scalar use");
        // batch letter: a free letter of the block; rotate it to the first position
        std::string key = jl;
        for (auto& kv : P.space) key += std::string(1, kv.first) + kv.second;
        pppp[key].push_back(&P);
        continue;
      }
      plain.push_back({pidx, &P});
    }
    if (plain.empty()) {
      // only (PP|PP) products
    } else if (grouped && run_grouped(plain, outs, scalar_out)) {
      ++grouped_uses;
    } else if (grouped) {
      // too large to group as a whole: the small products run grouped in waves whose
      // temporaries fit, the others one launch each; scalar uses sum the waves' partial
      // values in a fixed order
      std::vector<std::pair<int, const TProduct*>> large;
      std::vector<std::vector<std::pair<int, const TProduct*>>> waves(1);
      double wave_bytes = 0;
      for (auto& pp : plain) {
        double temp = 0, flops = 0;
        product_cost(*pp.second, temp, flops);
        if (temp * 8 > kSmallProductBytes || flops > kSmallProductFlops) {
          large.push_back(pp);
          continue;
        }
        if (!waves.back().empty() && wave_bytes + temp * 8 > 0.75 * group_cap) {
          waves.emplace_back();
          wave_bytes = 0;
        }
        waves.back().push_back(pp);
        wave_bytes += temp * 8;
      }
      const int nw = (int)waves.size();
      double* part = scalar_out ? pool.alloc(nw + 1) : nullptr;
      for (int w = 0; w < nw; ++w) {
        double* pw = part ? part + w : nullptr;
        if (run_grouped(waves[w], outs, pw)) ++grouped_uses;
        else run_serial(waves[w], outs, pw);
      }
      run_serial(large, outs, part ? part + nw : nullptr);
      if (scalar_out) {
        double* ones = upload(std::vector<double>(nw + 1, 1.0));
        op([nw, part, ones, scalar_out](hipStream_t s) { launch_weighted_sum(nw + 1, part, ones, scalar_out, s); });
      }
    } else {
      run_serial(plain, outs, scalar_out);
    }
    for (auto& grp : pppp) {
      const TProduct& P0 = *grp.second[0];
      std::string L, key;
      for (auto& f : P0.f)
        if (f.tensor == "J") canon_j(f.letters, P0.space, L, key);
      // the first letter of the canonical block must be free in every product of the group
      char bl = 0;
      for (int k = 0; k < 4 && !bl; ++k) {
        bool free_all = true;
        for (auto* P : grp.second)
          if (P->res.find(L[k]) == std::string::npos) free_all = false;
        if (free_all) bl = L[k];
      }
      if (!bl) throw Error(DSRG_E_HIP, "internal: no free letter to batch the (PP|PP) block");
      const int nP = d.len('P'), nH = d.len('H');
      const int lbl = d.len(P0.space.at(bl));
      // products on unique index pairs, one contraction per distinct amplitude array and part
      std::vector<const TProduct*> full;
      std::vector<const double*> pt[3];
      std::vector<std::vector<LadderTarget>> po[3];
      std::vector<LadderTarget> tg;
      for (auto* P : grp.second) {
        const double* Tt = nullptr;
        const int kind = (nP > 0 && nH > 0) ? pair_ladder(*P, bl, outs, Tt, tg) : 0;
        if (!kind) {
          full.push_back(P);
          continue;
        }
        size_t k = std::find(pt[kind].begin(), pt[kind].end(), Tt) - pt[kind].begin();
        if (k == pt[kind].size()) {
          pt[kind].push_back(Tt);
          po[kind].emplace_back();
        }
        po[kind][k].insert(po[kind][k].end(), tg.begin(), tg.end());
      }
      const bool pairs = !pt[1].empty() || !pt[2].empty();
      const bool sym = !pt[2].empty();
      // with every product on unique pairs the batch holds the rows q >= b0 only
      const bool tri_build = pairs && full.empty();
      const long long kp = (long long)nP * (nP - 1) / 2, kp1 = kp + nP;
      const long long np = (long long)nH * (nH - 1) / 2, np1 = np + nH;
      // The whole (PP|PP) block over particle pairs x <= y, K[pair(p, x)][pair(q, y)] =
      // (p x|q y), resident when it fits the workspace beside one value's packed rows: one
      // triangular contraction over the packed B builds it (the pair symmetries of real
      // integrals leave a quarter of the batched build's work) and the pair packs read it.
      const long long npk = (long long)nP * (nP + 1) / 2;
      const long long per_rows = pairs ? (long long)nP * (kp + (sym ? kp1 : 0)) : 0;
      const long long kbytes = 8 * (npk * npk + (long long)M * npk);   // K and the packed B
      bool fullk = tri_build && per_rows > 0 && npk < (1LL << 31) && ws_cap - kbytes >= 8 * per_rows;
      if (fullk && virt_batch > 0 &&
          (ws_cap - kbytes) / (8 * per_rows) < std::min<long long>(virt_batch, lbl))
        fullk = false;   // the requested batch needs the batched build's memory
      // doubles per value of the batch letter: integral rows (batched build) plus packed rows
      const long long per = (long long)nP * nP * nP;
      const long long per_all = (fullk ? 0 : per) + per_rows;
      const long long fit = (ws_cap - (fullk ? kbytes : 0)) / (8 * per_all);
      if (fit < 1)
        throw Error(DSRG_E_OOM, "workspace_cap of " + std::to_string(ws_cap) + " bytes is below one (PP|PP) batch row of " +
                                    std::to_string(8 * per_all) + " bytes");
      long long nb = std::min<long long>(lbl, virt_batch > 0 ? (long long)virt_batch : fit);
      if (nb > fit)
        throw Error(DSRG_E_OOM, "virt_batch " + std::to_string(virt_batch) + " needs " + std::to_string(8 * per_all * nb) +
                                    " bytes, above workspace_cap");
      ladder_batch = (int)nb;
      // pair tables: strict pairs (m = own index) and pairs a <= b (m = strict index or -1),
      // p-major row lists with the first row of each p
      auto pairs_of = [](int n, bool diag, std::vector<LadderPair>& v, std::vector<long long>* start) {
        int m = 0;
        for (int a = 0; a < n; ++a) {
          if (start) start->push_back((long long)v.size());
          for (int b = diag ? a : a + 1; b < n; ++b) v.push_back({a, b, b > a ? m++ : -1});
        }
        if (start) start->push_back((long long)v.size());
      };
      std::vector<long long> rs0, rs1;
      LadderPair *rows0 = nullptr, *rows1 = nullptr, *kt0 = nullptr, *kt1 = nullptr, *nt0 = nullptr,
                 *nt1 = nullptr;
      // packed amplitudes: the parts that multiply the antisymmetrised rows (same-spin
      // amplitudes, then the antisymmetric parts of the opposite-spin ones) side by side in
      // one [na_t * np][kp] operand, so one contraction serves them all; the symmetric
      // parts [np1][kp1] each
      std::vector<double*> tpk2;
      double* Tanti = nullptr;
      const long long na_t = (long long)pt[1].size() + (long long)pt[2].size();
      const long long ldx = na_t * np;
      double *Va = nullptr, *Vs = nullptr, *Xa = nullptr, *Xs = nullptr;
      auto pack_t = [&](const double* Tt, const LadderPair* kt, long long k, const LadderPair* nt, long long n,
                        int mode, double* into) {
        double* tp = into ? into : pool.alloc((size_t)std::max(1LL, k * n));
        const int nPl = nP, nHl = nH, ki = (int)k, ni = (int)n;
        op([Tt, nPl, nHl, kt, ki, nt, ni, mode, tp](hipStream_t s) {
          launch_ladder_pack_t(Tt, nPl, nHl, kt, ki, nt, ni, mode, tp, s);
        });
        ++n_launch;
        return tp;
      };
      if (pairs) {
        if (P0.space.at(bl) != 'P') throw Error(DSRG_E_HIP, "internal: ladder batch letter outside P");
        if (kp1 >= (1LL << 31) || (long long)nb * nP * std::max(nP, nH) >= (1LL << 31))
          throw Error(DSRG_E_UNSUPPORTED, "ladder pair contraction dimension exceeds 2^31");
        std::vector<LadderPair> r0, r1, k0, k1, n0, n1v;
        pairs_of(nP, false, r0, &rs0);
        pairs_of(nP, false, k0, nullptr);
        pairs_of(nH, false, n0, nullptr);
        rows0 = upload(r0);
        kt0 = upload(k0);
        nt0 = upload(n0);
        if (sym) {
          pairs_of(nP, true, r1, &rs1);
          pairs_of(nP, true, k1, nullptr);
          pairs_of(nH, true, n1v, nullptr);
          rows1 = upload(r1);
          kt1 = upload(k1);
          nt1 = upload(n1v);
        }
        long long mr0 = 0, mr1 = 0;
        for (int b0 = 0; b0 < nP; b0 += (int)nb) {
          const int b1 = (int)std::min<long long>(nP, b0 + nb);
          mr0 = std::max(mr0, rs0[b1] - rs0[b0]);
          if (sym) mr1 = std::max(mr1, rs1[b1] - rs1[b0]);
        }
        Va = pool.alloc((size_t)std::max(1LL, mr0 * kp));
        Xa = pool.alloc((size_t)std::max(1LL, mr0 * ldx));
        if (sym) {
          Vs = pool.alloc((size_t)std::max(1LL, mr1 * kp1));
          Xs = pool.alloc((size_t)std::max(1LL, mr1 * np1));
        }
        if (kp > 0 && np > 0) {
          Tanti = pool.alloc((size_t)std::max(1LL, ldx * kp));
          long long j = 0;
          for (const double* Tt : pt[1]) pack_t(Tt, kt0, kp, nt0, np, 0, Tanti + (j++) * np * kp);
          for (const double* Tt : pt[2]) pack_t(Tt, kt0, kp, nt0, np, 2, Tanti + (j++) * np * kp);
        }
        for (const double* Tt : pt[2]) tpk2.push_back(pack_t(Tt, kt1, kp1, nt1, np1, 1, nullptr));
      }
      // C[row][n] = sum_k A[row][k] B[n][k]
      auto pair_gemm = [&](const double* A, const double* Bm, double* C, long long rows, long long n,
                           long long k) {
        GettDesc g;
        g.nm = 1; g.nn = 1; g.nk = 1;
        g.md[0] = (int)rows; g.nd[0] = (int)n; g.kd[0] = (int)k;
        g.M = (int)rows; g.N = (int)n; g.K = (int)k;
        g.am[0] = k; g.ak[0] = 1;
        g.bn[0] = k; g.bk[0] = 1;
        g.cm[0] = n; g.cn[0] = 1;
        g.alpha = 1.0; g.beta = 0;
        gett_prepare(g);
        gett(g, A, Bm, C, kRoleLadder);
      };
      // products are written with the batch letter first in the J factor: rotate letters
      double* jb = fullk ? nullptr : jbatch_buffer(nb * per);
      double* Kfull = nullptr;
      if (fullk) {
        double* Bp = pool.alloc((size_t)M * npk);
        const int Nl = d.nC + d.nA + d.nV, offP = d.off('P'), nPl = nP, Ml = M;
        const double* Bl = B;
        op([Bl, Nl, offP, nPl, Ml, Bp](hipStream_t s) { launch_pack_pairs(Bl, Nl, offP, nPl, Ml, Bp, s); });
        ++n_launch;
        Kfull = pool.alloc((size_t)(npk * npk));
        GettDesc g;
        g.nm = 1; g.nn = 1; g.nk = 1;
        g.md[0] = (int)npk; g.nd[0] = (int)npk; g.kd[0] = M;
        g.M = (int)npk; g.N = (int)npk; g.K = M;
        g.am[0] = 1; g.ak[0] = npk;
        g.bk[0] = npk; g.bn[0] = 1;
        g.cm[0] = npk; g.cn[0] = 1;
        g.alpha = 1.0; g.beta = 0;
        gett_prepare(g);
        g.tri = kFullKBlock;   // the blocks below the diagonal are mirrored instead
        double fb0 = gett_flops;
        gett(g, Bp, Bp, Kfull, kRoleIntegrals);
        ladder_flops += gett_flops - fb0;
        double* Kl = Kfull;
        const long long nk = npk;
        op([Kl, nk](hipStream_t s) { launch_mirror_lower(Kl, nk, kFullKBlock, s); });
        ++n_launch;
      }
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (profile) {
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, st));
      }
      for (int b0 = 0; b0 < lbl; b0 += (int)nb) {
        int n1 = (int)std::min<long long>(nb, lbl - b0);
        // J(P P | P P) batch with the first index in [b0, b0+n1) of the batch letter's space
        // and the third in [qoff, nP)
        int off1 = d.off(P0.space.at(bl)) - d.off('P') + b0;
        const int qoff = tri_build ? b0 : 0, nq = nP - qoff;
        double fb = gett_flops;
        // with rows q >= b0 only, the blocks of rows p and columns q < p stay unbuilt (the
        // packs read q >= p)
        if (!fullk) build_j('P', 'P', 'P', 'P', off1, n1, jb, qoff, nq, tri_build ? nP : 0);
        const double* Kl = Kfull;
        if (pairs) {
          const long long r0 = rs0[b0], na = rs0[b0 + n1] - r0;
          const long long s0 = sym ? rs1[b0] : 0, ns = sym ? rs1[b0 + n1] - s0 : 0;
          const LadderPair* ra = rows0 + r0;
          const LadderPair* rsy = sym ? rows1 + s0 : nullptr;
          const int nPl = nP, nHl = nH, nai = (int)na, nsi = (int)ns;
          const int npi = (int)np, np1i = (int)np1, m0 = (int)r0, ldxi = (int)ldx;
          const bool anti_part = na > 0 && kp > 0 && np > 0;
          if (anti_part && ns > 0) {
            // both parts from one read of the batch: the rows p <= q carry the strict ones
            const long long r0l = r0;
            op([jb, Kl, nPl, b0, qoff, nq, rsy, nsi, Vs, Va, r0l](hipStream_t s) {
              if (Kl) launch_ladder_pack_vk(Kl, nPl, rsy, nsi, 1, Vs, s, Va, r0l);
              else launch_ladder_pack_v(jb, nPl, b0, qoff, nq, rsy, nsi, 1, Vs, s, Va, r0l);
            });
            ++n_launch;
          } else {
            if (anti_part) {
              op([jb, Kl, nPl, b0, qoff, nq, ra, nai, Va](hipStream_t s) {
                if (Kl) launch_ladder_pack_vk(Kl, nPl, ra, nai, 0, Va, s);
                else launch_ladder_pack_v(jb, nPl, b0, qoff, nq, ra, nai, 0, Va, s);
              });
              ++n_launch;
            }
            if (ns > 0) {
              op([jb, Kl, nPl, b0, qoff, nq, rsy, nsi, Vs](hipStream_t s) {
                if (Kl) launch_ladder_pack_vk(Kl, nPl, rsy, nsi, 1, Vs, s);
                else launch_ladder_pack_v(jb, nPl, b0, qoff, nq, rsy, nsi, 1, Vs, s);
              });
              ++n_launch;
            }
          }
          role_now = kRoleLadder;
          // Xa[row][j np + n]: block j of every antisymmetric part in one contraction
          if (anti_part) pair_gemm(Va, Tanti, Xa, na, ldx, kp);
          if (anti_part)
            for (size_t k = 0; k < pt[1].size(); ++k) {
              const double* Xk = Xa + (long long)k * np;
              for (auto& tg : po[1][k]) {
                double* Ot = tg.O;
                const double c = tg.c;
                op([Xk, nai, npi, ldxi, ra, nt0, nPl, nHl, c, Ot](hipStream_t s) {
                  launch_ladder_unpack_anti(Xk, nai, npi, ldxi, ra, nt0, nPl, nHl, c, Ot, s);
                });
                ++n_launch;
              }
            }
          if (ns > 0)
            for (size_t k = 0; k < pt[2].size(); ++k) {
              const double* Xk = Xa + (long long)(pt[1].size() + k) * np;
              pair_gemm(Vs, tpk2[k], Xs, ns, np1, kp1);
              for (auto& tg : po[2][k]) {
                double* Ot = tg.O;
                const double c = tg.c;
                op([Xs, Xk, nsi, np1i, ldxi, m0, rsy, nt1, nPl, nHl, c, Ot](hipStream_t s) {
                  launch_ladder_unpack_sym(Xs, Xk, nsi, np1i, ldxi, m0, rsy, nt1, nPl, nHl, c, Ot, s);
                });
                ++n_launch;
              }
            }
          role_now = kRoleGeneric;
        }
        for (auto* P : full) {
          TProduct Q = *P;
          for (auto& f : Q.f)
            if (f.tensor == "J") f.letters = rotate_first(f.letters, bl, Q.space);
          LetterRange lr = full_range(Q);
          lr.off[bl] = b0;
          lr.len[bl] = n1;
          double c = 0;
          role_now = kRoleLadder;
          run_product(Q, lr, jb, bl, outs, nullptr, c, 0.0);
          role_now = kRoleGeneric;
        }
        ladder_flops += gett_flops - fb;  // integral batch build plus the ladder products
      }
      if (profile) {
        HIPCHECK(hipEventRecord(e1, st));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        ladder_ms += ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
      }
    }
  }

  // (PP|PP) batch buffer, shared by the ladder groups of the call (stream order makes the
  // reuse safe)
  double* jb_buf = nullptr;
  long long jb_cap = 0;
  double* jbatch_buffer(long long n) {
    if (n > jb_cap) {
      if (jb_buf) pool.release(jb_buf);
      jb_buf = pool.alloc((size_t)n);
      jb_cap = n;
    }
    return jb_buf;
  }

  // Rewrite J(l1 l2|l3 l4) so that letter bl comes first (symmetries of real (pr|qs)).
  static std::string rotate_first(const std::string& L0, char bl, const std::map<char, char>& sp) {
    std::string L, key;
    canon_j(L0, sp, L, key);
    if (L[0] == bl) return L;
    if (L[1] == bl) return std::string() + L[1] + L[0] + L[2] + L[3];
    if (L[2] == bl) return std::string() + L[2] + L[3] + L[0] + L[1];
    return std::string() + L[3] + L[2] + L[0] + L[1];
  }
};

// ---------------------------------------------------------------------------
// Pipeline
// ---------------------------------------------------------------------------
// Errors from the device-side input counters: non-finite values first, then densities.
static void check_bad(const int* bad) {
  if (bad[0]) throw Error(DSRG_E_NONFINITE, "non-finite value in eps, B, f_offdiag or the densities");
  if (bad[1]) throw Error(DSRG_E_RDM, "gamma1 not symmetric or gamma2 not Hermitian/antisymmetric");
}

static bool finite_host(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Device inputs: every array copied into the library's buffers by one launch, which also
// counts non-finite values (one launch instead of a copy and a check per array).
struct CopyList {
  const double* src[6];
  double* dst[6];
  long long end[6];   // prefix sums of the array lengths
  int n;
};

// Reference densities as the ABI requires them (Sec. II.A: real densities of one state):
// gamma1 symmetric, gamma2 Hermitian (uv <-> xy) and, in its same-spin blocks,
// antisymmetric in u <-> v and in x <-> y; violations beyond kRdmTol are counted.
constexpr double kRdmTol = 1e-10;
__host__ __device__ inline int rdm_violations(int nA, const double* g1, const double* g2, long long e) {
  const long long n2 = (long long)nA * nA, n4 = n2 * n2;
  if (e < 2 * n2) {
    const long long s = e / n2, r = e - s * n2, u = r / nA, v = r - u * nA;
    return fabs(g1[s * n2 + u * nA + v] - g1[s * n2 + v * nA + u]) > kRdmTol;
  }
  e -= 2 * n2;
  if (e >= 3 * n4) return 0;
  const long long b = e / n4, r = e - b * n4;
  const long long u = r / (n2 * nA), v = (r / n2) % nA, x = (r / nA) % nA, y = r % nA;
  const double* g = g2 + b * n4;
  const double val = g[r];
  int bad = fabs(val - g[x * n2 * nA + y * n2 + u * nA + v]) > kRdmTol;
  if (b != 1) {
    bad += fabs(val + g[v * n2 * nA + u * n2 + x * nA + y]) > kRdmTol;
    bad += fabs(val + g[u * n2 * nA + v * n2 + y * nA + x]) > kRdmTol;
  }
  return bad;
}
__global__ __launch_bounds__(256) void rdm_check_kernel(int nA, const double* __restrict__ g1,
                                                        const double* __restrict__ g2, int* __restrict__ bad) {
  const long long n2 = (long long)nA * nA, total = 2 * n2 + 3 * n2 * n2;
  int nbad = 0;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x)
    nbad += rdm_violations(nA, g1, g2, e);
  if (nbad) atomicAdd(bad + 1, nbad);
}
__global__ __launch_bounds__(256) void copy_check_kernel(CopyList L, int* __restrict__ bad) {
  const long long total = L.end[L.n - 1];
  int nbad = 0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < total; i += 256LL * gridDim.x) {
    int k = 0;
    while (k + 1 < L.n && i >= L.end[k]) ++k;
    const long long j = i - (k ? L.end[k - 1] : 0);
    const double v = L.src[k][j];
    L.dst[k][j] = v;
    nbad += !isfinite(v);
  }
  if (nbad) atomicAdd(bad, nbad);
}

// Shape of a call and the device copies of its inputs.  The pipeline reads only these
// copies (and s from device memory), so a graph captured once serves every later call of
// the same shape, whatever the input values, s and input pointers.
struct Shape {
  int nC, nA, nV, M;
  bool has_g3, pt3, has_f = false;
  long long N, nB, g1n, g2n, g3n;
};

struct Inputs {
  double *eps = nullptr, *B = nullptr, *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;
  double* f = nullptr;         // [N][N] inter-block Fock elements (with f_offdiag)
  double* s = nullptr;         // [1]
  double* energies = nullptr;  // [4]: E(2), E(3)_a, E(3)_b, unused
  int* bad = nullptr;          // [2]: non-finite values, density violations (device inputs)
};

static Inputs alloc_inputs(Pool& pool, const Shape& sh) {
  Inputs in;
  in.eps = pool.alloc((size_t)sh.N);
  in.B = pool.alloc((size_t)sh.nB);
  if (sh.nA > 0) {
    in.g1 = pool.alloc((size_t)sh.g1n);
    in.g2 = pool.alloc((size_t)sh.g2n);
  }
  if (sh.has_g3) in.g3 = pool.alloc((size_t)sh.g3n);
  if (sh.has_f) in.f = pool.alloc((size_t)(sh.N * sh.N));
  in.s = pool.alloc(1);
  in.energies = pool.alloc(4);
  in.bad = (int*)pool.alloc(1);
  return in;
}

// Copy the inputs into the device buffers (host or device sources) and s from s_host,
// which must stay valid until the stream is synchronised.  Device inputs are checked for
// non-finite values on the copies (one synchronisation).
// With defer_bad (pinned host memory) the non-finite count of device inputs is only copied
// there, and the caller checks it after its own synchronisation (no wait here).
static void load_inputs(const dsrg_problem* P, bool devptr, const Shape& sh, const Inputs& in,
                        const double* s_host, hipStream_t st, int* defer_bad = nullptr) {
  HIPCHECK(hipMemcpyAsync(in.s, s_host, sizeof(double), hipMemcpyHostToDevice, st));
  if (!devptr) {
    auto cp = [&](double* dst, const double* src, long long n) {
      if (n > 0) HIPCHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st));
    };
    cp(in.eps, P->eps, sh.N);
    cp(in.B, P->B, sh.nB);
    if (sh.nA > 0) {
      cp(in.g1, P->gamma1, sh.g1n);
      cp(in.g2, P->gamma2, sh.g2n);
    }
    if (sh.has_g3) cp(in.g3, P->gamma3, sh.g3n);
    if (sh.has_f) cp(in.f, P->f_offdiag, sh.N * sh.N);
    return;
  }
  // both counters in one double (a fill kernel rather than a memset node)
  launch_fill(reinterpret_cast<double*>(in.bad), 1, 0.0, st);
  CopyList L{};
  long long total = 0;
  auto add = [&](double* dst, const double* src, long long n) {
    if (n <= 0) return;
    L.src[L.n] = src;
    L.dst[L.n] = dst;
    total += n;
    L.end[L.n] = total;
    ++L.n;
  };
  add(in.eps, P->eps, sh.N);
  add(in.B, P->B, sh.nB);
  if (sh.nA > 0) {
    add(in.g1, P->gamma1, sh.g1n);
    add(in.g2, P->gamma2, sh.g2n);
  }
  if (sh.has_g3) add(in.g3, P->gamma3, sh.g3n);
  if (sh.has_f) add(in.f, P->f_offdiag, sh.N * sh.N);
  if (L.n > 0) {
    const long long blocks = std::min<long long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(copy_check_kernel, dim3((unsigned)blocks), dim3(256), 0, st, L, in.bad);
    HIPCHECK(hipGetLastError());
  }
  if (sh.nA > 0) {
    const long long n2 = (long long)sh.nA * sh.nA, total_r = 2 * n2 + 3 * n2 * n2;
    const long long blocks = std::min<long long>((total_r + 255) / 256, 1024);
    hipLaunchKernelGGL(rdm_check_kernel, dim3((unsigned)blocks), dim3(256), 0, st, sh.nA, in.g1, in.g2, in.bad);
    HIPCHECK(hipGetLastError());
  }
  if (defer_bad) {
    HIPCHECK(hipMemcpyAsync(defer_bad, in.bad, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    return;
  }
  int hbad[2] = {0, 0};
  HIPCHECK(hipMemcpyAsync(hbad, in.bad, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  check_bad(hbad);
}

// Stage marks of the pipeline (ev null: no stage timing, as in the allocation-free entry).
static void mark(hipEvent_t* ev, int k, hipStream_t st) {
  if (ev) HIPCHECK(hipEventRecord(ev[k], st));
}

// Device buffers of the intermediates a caller may ask for.
struct BodyOut {
  double *T1a = nullptr, *T1b = nullptr, *T2aa = nullptr, *T2ab = nullptr;
  double *W1 = nullptr, *W2 = nullptr, *Z1 = nullptr, *Z2 = nullptr, *U1 = nullptr, *U2 = nullptr;
  double* pairs = nullptr;   // [nC (nC + 1) / 2 + 1]: core-pair parts of E(3), then the rest
  // with relax: active blocks R1 [2][nA][nA], R2 [3][nA]^4 of [H~(1), A(1)] + [H~(2)_{1,2}, A(1)]
  // + [H~(1), A(2)] (twice the active blocks of Hbar^(2) + Hbar^(3), Eqs. Hbar_2nd, Hbar_3rd)
  double* R = nullptr;
};

// A use with its factor tensors renamed (the same products on other arrays).
static Use rename_use(const Use& U, const char* from1, const char* to1, const char* from2, const char* to2) {
  Use u = U;
  for (auto& P : u)
    for (auto& f : P.f) {
      if (f.tensor == from1) f.tensor = to1;
      else if (f.tensor == from2) f.tensor = to2;
    }
  return u;
}

// The pipeline: every device operation goes through op (and so into a plan being built);
// ev[1..6] mark the stages on st.
// The pipeline modes: PairsMode runs the core-pair decomposition of E(3) beside the plain
// energies; RestMode computes E(2) and only the rest of E(3) (the parts of the
// decomposition outside the core pairs, from the restricted uses of [V, A(1)] and
// [Y, A(1)] and first-order doubles without their core-core pairs) plus the features of
// the core pairs.
enum BodyMode { PlainMode = 0, PairsMode = 1, RestMode = 2 };
struct RestOut {
  float* feat = nullptr;   // [nC (nC + 1) / 2][16] device
  double* e2 = nullptr;    // [nC (nC + 1) / 2] device
};

static BodyOut body(Exec& X, OpLog& op, Pool& pool, const Shape& sh, const Inputs& in, hipEvent_t* ev,
                    hipStream_t st, bool want_pairs = false, RestOut* rest = nullptr, bool relax = false) {
  const int nC = sh.nC, nA = sh.nA, nV = sh.nV;
  const int nH = nC + nA, nP = nA + nV;
  const Dims d{nC, nA, nV};
  const double *eps = in.eps, *g1 = in.g1, *g2 = in.g2, *g3 = in.g3, *sdev = in.s;
  BodyOut bo;
  // step a0: spin-orbital densities and cumulants over the active space
  const int n2 = 2 * nA;
  if (nA > 0) {
    const long long e2n = (long long)n2 * n2, e4n = e2n * e2n, e6n = e4n * e2n;
    double* G1 = pool.alloc((size_t)e2n);
    double* G2 = pool.alloc((size_t)e4n);
    double* L2 = pool.alloc((size_t)e4n);
    double* eta = pool.alloc((size_t)e2n);
    double* L3 = pool.alloc((size_t)e6n);
    op([nA, g1, G1, g2, G2](hipStream_t s) { launch_expand_rdm12(nA, g1, G1, g2, G2, s); });
    if (g3) {
      // the spin blocks of gamma3 go straight into the three-body cumulant
      op([nA, g3, G1, G2, L2, L3, eta](hipStream_t s) { launch_cumulants(nA, G1, G2, g3, L2, L3, eta, s); });
    } else {
      op([nA, G1, G2, L2, eta](hipStream_t s) { launch_cumulants(nA, G1, G2, nullptr, L2, nullptr, eta, s); });
      op([L3, e6n](hipStream_t s) { launch_fill(L3, e6n, 0.0, s); });
    }
    pool.release(G2);
    // spin-block views of the spin-orbital arrays
    long long s1 = 1, s2 = n2, s3 = (long long)n2 * n2, s4 = s3 * n2, s5 = s4 * n2, s6 = s5 * n2;
    X.set_view("gA.a", G1, "AA", {s2, s1}, s3);
    X.set_view("gA.b", G1 + nA * s2 + nA, "AA", {s2, s1}, s3 - nA * s2 - nA);
    X.set_view("eA.a", eta, "AA", {s2, s1}, s3);
    X.set_view("eA.b", eta + nA * s2 + nA, "AA", {s2, s1}, s3 - nA * s2 - nA);
    std::vector<long long> st4{s4, s3, s2, s1}, st6{s6, s5, s4, s3, s2, s1};
    auto off = [&](std::vector<int> spins, std::vector<long long>& strd) {
      long long o = 0;
      for (size_t k = 0; k < spins.size(); ++k) o += spins[k] * nA * strd[k];
      return o;
    };
    X.set_view("L2.aa", L2 + off({0, 0, 0, 0}, st4), "AAAA", st4, s5 - off({0, 0, 0, 0}, st4));
    X.set_view("L2.ab", L2 + off({0, 1, 0, 1}, st4), "AAAA", st4, s5 - off({0, 1, 0, 1}, st4));
    X.set_view("L2.bb", L2 + off({1, 1, 1, 1}, st4), "AAAA", st4, s5 - off({1, 1, 1, 1}, st4));
    X.set_view("L3.aaa", L3 + off({0, 0, 0, 0, 0, 0}, st6), "AAAAAA", st6, s6 * n2 - off({0, 0, 0, 0, 0, 0}, st6));
    X.set_view("L3.aab", L3 + off({0, 0, 1, 0, 0, 1}, st6), "AAAAAA", st6, s6 * n2 - off({0, 0, 1, 0, 0, 1}, st6));
    X.set_view("L3.abb", L3 + off({0, 1, 1, 0, 1, 1}, st6), "AAAAAA", st6, s6 * n2 - off({0, 1, 1, 0, 1, 1}, st6));
    X.set_view("L3.bbb", L3 + off({1, 1, 1, 1, 1, 1}, st6), "AAAAAA", st6, s6 * n2 - off({1, 1, 1, 1, 1, 1}, st6));
  }
  // Coulomb blocks used by the first-order amplitudes
  {
    // every Coulomb block the tables read, except the batched (PP|PP) one
    std::vector<std::string> keys{"HPHP"};
    for (const char* u : {"C0", "W", "Z"})
      for (const TProduct& P : table().at(u))
        for (auto& f : P.f)
          if (f.tensor == "J") {
            std::string L, key;
            Exec::canon_j(f.letters, P.space, L, key);
            if (key != "PPPP") keys.push_back(key);
          }
    X.prebuild_j(keys);
  }
  double* Jhphp = X.jblock("HPHP");
  mark(ev, 1, st);

  // step a2: first-order amplitudes, Y = [H(0), A(1)] and H~(1) (excitation blocks)
  const size_t n4 = (size_t)nP * nP * nH * nH, n1 = (size_t)nP * nH;
  const AmpDims ad{nC, nA, nV};
  double* T2aa = pool.alloc(n4); double* T2ab = pool.alloc(n4);
  double* Y2aa = pool.alloc(n4); double* Y2ab = pool.alloc(n4);
  double* E2aa = pool.alloc(n4); double* E2ab = pool.alloc(n4);
  op([=](hipStream_t s) {
    launch_first_order_doubles(ad, Jhphp, eps, sdev, T2aa, T2ab, Y2aa, Y2ab, E2aa, E2ab, s);
  });
  double* T1a = pool.alloc(n1); double* T1b = pool.alloc(n1);
  double* Y1a = pool.alloc(n1); double* Y1b = pool.alloc(n1);
  // gamma1 input blocks [2][nA][nA] are read directly by the singles kernel
  const double* g1a = nA > 0 ? g1 : nullptr;
  const double* g1b = nA > 0 ? g1 + nA * nA : nullptr;
  // inter-block Fock elements f(1) (H(1) = f(1) + V): they drive the singles (Eq. T1_1st),
  // H~(1) = 2 H(1) + Y gains 2 f(1) in its one-body part, and O1 gains 2 [f(1), A(1)]
  double* F1 = nullptr;
  if (sh.has_f) {
    F1 = pool.alloc(n1);
    const double* fin = in.f;
    op([=](hipStream_t s) { launch_fock_exc(ad, fin, F1, s); });
  }
  // the singles launch writes the source (f + coup) exp(-s D^2), which is Y1 + f(1)
  op([=](hipStream_t s) {
    launch_singles(ad, T2aa, T2ab, T2aa, g1a, g1b, eps, sdev, F1, F1, T1a, T1b, Y1a, Y1b, s);
  });
  double *E1a = Y1a, *E1b = Y1b;
  if (F1) {
    // Y1 = source - f(1), H~(1) one-body = source + f(1)
    E1a = pool.alloc(n1);
    E1b = pool.alloc(n1);
    op([=](hipStream_t s) {
      launch_split_source((long long)n1, 1, Y1a, E1a, F1, s);
      launch_split_source((long long)n1, 1, Y1b, E1b, F1, s);
    });
  }
  auto bind_first = [&]() {
    X.set("T1.a", T1a, "PH"); X.set("T1.b", T1b, "PH");
    // first-order doubles: regularised integrals, so the same-spin blocks are antisymmetric
    // and the opposite-spin block is symmetric under the exchange of both pairs
    X.set("T2.aa", T2aa, "PPHH", 1); X.set("T2.ab", T2ab, "PPHH", 2); X.set("T2.bb", T2aa, "PPHH", 1);
  };
  bind_first();
  X.set("E1.a", E1a, "PH"); X.set("E1.b", E1b, "PH");
  X.set("E2.aa", E2aa, "PPHH"); X.set("E2.ab", E2ab, "PPHH"); X.set("E2.bb", E2aa, "PPHH");
  X.set("Y1.a", Y1a, "PH"); X.set("Y1.b", Y1b, "PH");
  X.set("Y2.aa", Y2aa, "PPHH"); X.set("Y2.ab", Y2ab, "PPHH"); X.set("Y2.bb", Y2aa, "PPHH");
  bo.T1a = T1a; bo.T1b = T1b; bo.T2aa = T2aa; bo.T2ab = T2ab;
  mark(ev, 2, st);
  if (rest && nC > 0) {
    const int npairs = nC * (nC + 1) / 2;
    rest->feat = reinterpret_cast<float*>(pool.alloc((size_t)npairs * 8));   // 16 floats per pair
    rest->e2 = pool.alloc((size_t)npairs);
    float* feat = rest->feat;
    double* e2p = rest->e2;
    const double* Bd = in.B;
    const int Maux = sh.M;
    op([=](hipStream_t s) { launch_pair_features(ad, Jhphp, eps, sdev, Bd, Maux, feat, e2p, s); });
  }

  auto& T = table();
  const Use& C0 = T.at("C0");
  double* energies = in.energies;
  op([energies](hipStream_t s) { launch_fill(energies, 4, 0.0, s); });
  std::map<std::string, TensorRef> none;
  auto scalar = [&](double* outp) {
    X.use_id = 0;
    X.run_use(C0, none, outp);
  };
  if (!sh.pt3) {
    // step a3: E(2) = <[H~(1), T(1)]>
    scalar(energies + 0);
    for (int k = 3; k < 7; ++k) mark(ev, k, st);
    return bo;
  }
  // W = [V, A(1)]_{1,2} and Z = [Y, A(1)]_{1,2}, excitation blocks
  // one zeroed block: W one-body, W two-body, Z one-body, Z two-body
  const long long wz = 2 * (2 * (long long)n1 + 3 * (long long)n4);
  double* W1 = pool.alloc((size_t)wz);
  double* W2 = W1 + 2 * n1;
  double* Z1 = W2 + 3 * n4;
  double* Z2 = Z1 + 2 * n1;
  op([W1, wz](hipStream_t s) { launch_fill(W1, wz, 0.0, s); });
  auto bind_out = [&](std::map<std::string, TensorRef>& o, double* p1, double* p2) {
    auto mk = [&](double* p, const char* ax) {
      TensorRef t{p, ax, {}};
      int r = (int)strlen(ax);
      t.stride.assign(r, 1);
      for (int k = r - 2; k >= 0; --k) t.stride[k] = t.stride[k + 1] * d.len(ax[k + 1]);
      t.lim = t.stride[0] * d.len(ax[0]);
      return t;
    };
    o["O1.a"] = mk(p1, "PH"); o["O1.b"] = mk(p1 + n1, "PH");
    o["O2.aa"] = mk(p2, "PPHH"); o["O2.ab"] = mk(p2 + n4, "PPHH"); o["O2.bb"] = mk(p2 + 2 * n4, "PPHH");
  };
  std::map<std::string, TensorRef> wout, zout;
  bind_out(wout, W1, W2);
  bind_out(zout, Z1, Z2);
  // E(2), W and Z read only first-order quantities: for small problems (a doubles block of
  // at most 2^22 elements) one grouped run covers all three, with the stage time reported
  // under E(2); else step a3, steps a4-a5 and step a6 in turn
  std::map<std::string, TensorRef> none_e;
  X.use_id = 0;
  static const Use rest_w = rest_use(T.at("W")), rest_z = rest_use(T.at("Z"));
  const Use& Wu = rest ? rest_w : T.at("W");
  const Use& Zu = rest ? rest_z : T.at("Z");
  if ((long long)n4 <= (1LL << 22) &&
      X.run_fused({&C0, &Wu, &Zu}, {&none_e, &wout, &zout}, {energies + 0, nullptr, nullptr})) {
    for (int k = 3; k < 6; ++k) mark(ev, k, st);
  } else {
    scalar(energies + 0);
    mark(ev, 3, st);
    X.use_id = 1;
    X.run_use(Wu, wout, nullptr);
    mark(ev, 4, st);
    X.use_id = 2;
    X.run_use(Zu, zout, nullptr);
    mark(ev, 5, st);
  }
  if (F1) {
    // [f(1), A(1)]_{1,2}: the products of [Y, A(1)] with a one-body Y factor, with f(1) in its
    // place (both are Hermitian one-body operators with only excitation elements and their
    // adjoints), added into W, so that O1 = 2 (W + [f(1), A(1)]) + Z downstream
    Use fu;
    for (const TProduct& P : Zu) {
      bool one_body = false;
      for (auto& f : P.f) one_body = one_body || f.tensor == "Y1";
      if (!one_body) continue;
      TProduct Q = P;
      for (auto& f : Q.f)
        if (f.tensor == "Y1") f.tensor = "F1";
      fu.push_back(Q);
    }
    X.set("F1.a", F1, "PH"); X.set("F1.b", F1, "PH");
    const long long fwn = 2 * (long long)n1 + 3 * (long long)n4;
    double* FW = pool.alloc((size_t)fwn);
    op([FW, fwn](hipStream_t s) { launch_fill(FW, fwn, 0.0, s); });
    std::map<std::string, TensorRef> fout;
    bind_out(fout, FW, FW + 2 * n1);
    X.use_id = 5;
    X.run_use(fu, fout, nullptr);
    op([W1, FW, fwn](hipStream_t s) { launch_add(W1, FW, fwn, s); });   // W1, W2 are contiguous
  }
  // second-order amplitudes and H~(2)_{1,2}
  double* U2 = pool.alloc(3 * n4);
  double* H2 = pool.alloc(3 * n4);
  double* U1 = pool.alloc(2 * n1);
  double* S2 = pool.alloc(2 * n1);
  double* H1 = pool.alloc(2 * n1);
  op([=](hipStream_t s) {
    launch_second_order_doubles(ad, W2, Z2, eps, sdev, U2, H2, 3, s);   // aa, ab, bb
    // f(2) = W1 + Z1 / 2 formed inside the singles launch
    launch_singles(ad, U2, U2 + n4, U2 + 2 * n4, g1a, g1b, eps, sdev, W1, W1 + n1, U1, U1 + n1, S2,
                   S2 + n1, s, Z1, Z1 + n1);
    launch_second_order_h1(ad, W1, Z1, S2, H1, 2, s);   // alpha, beta
  });
  // One-step relaxation (Sec. II.B Eq. E_relaxed): the active blocks of the second- and
  // third-order transformed Hamiltonian, R = [H~(1), A(1)] + [H~(2)_{1,2}, A(1)] + [H~(1), A(2)]
  // (use R of the table on H~(1) or H~(2)_{1,2} as the de-excitation operator and either
  // order of amplitudes; Hbar^(2) + Hbar^(3) = R / 2 on the active blocks)
  auto relax_stage = [&]() {
    if (!relax || nA == 0) return;
    const long long n2 = (long long)nA * nA, nr = 2 * n2 + 3 * n2 * n2;
    double* R = pool.alloc((size_t)nr);
    op([R, nr](hipStream_t s) { launch_fill(R, nr, 0.0, s); });
    X.set("E1.a", E1a, "PH"); X.set("E1.b", E1b, "PH");
    X.set("E2.aa", E2aa, "PPHH"); X.set("E2.ab", E2ab, "PPHH"); X.set("E2.bb", E2aa, "PPHH");
    bind_first();
    X.set("U1.a", U1, "PH"); X.set("U1.b", U1 + n1, "PH");
    X.set("U2.aa", U2, "PPHH", 1); X.set("U2.ab", U2 + n4, "PPHH"); X.set("U2.bb", U2 + 2 * n4, "PPHH", 1);
    X.set("H1.a", H1, "PH"); X.set("H1.b", H1 + n1, "PH");
    X.set("H2.aa", H2, "PPHH"); X.set("H2.ab", H2 + n4, "PPHH"); X.set("H2.bb", H2 + 2 * n4, "PPHH");
    std::map<std::string, TensorRef> rout;
    auto mk = [&](double* p, const char* ax) {
      const int r = (int)strlen(ax);
      TensorRef t{p, ax, std::vector<long long>(r, 1)};
      for (int k = r - 2; k >= 0; --k) t.stride[k] = t.stride[k + 1] * nA;
      t.lim = t.stride[0] * nA;
      return t;
    };
    rout["R1.a"] = mk(R, "AA"); rout["R1.b"] = mk(R + n2, "AA");
    rout["R2.aa"] = mk(R + 2 * n2, "AAAA"); rout["R2.ab"] = mk(R + 2 * n2 + n2 * n2, "AAAA");
    rout["R2.bb"] = mk(R + 2 * n2 + 2 * n2 * n2, "AAAA");
    static const Use r_h2 = rename_use(T.at("R"), "E1", "H1", "E2", "H2");
    static const Use r_u = rename_use(T.at("R"), "T1", "U1", "T2", "U2");
    X.use_id = 6;
    X.run_use(T.at("R"), rout, nullptr);
    X.use_id = 7;
    X.run_use(r_h2, rout, nullptr);
    X.use_id = 8;
    X.run_use(r_u, rout, nullptr);
    bo.R = R;
  };
  // E(3)_a = <[H~(1), T(2)]> and E(3)_b = <[H~(2)_{1,2}, T(1)]>: without the pair
  // decomposition both scalars run as one grouped use when their temporaries fit (the
  // second-order tensors under their own names), else one after the other
  if (!want_pairs && !rest) {
    X.set("U1.a", U1, "PH"); X.set("U1.b", U1 + n1, "PH");
    X.set("U2.aa", U2, "PPHH", 1); X.set("U2.ab", U2 + n4, "PPHH"); X.set("U2.bb", U2 + 2 * n4, "PPHH", 1);
    X.set("H1.a", H1, "PH"); X.set("H1.b", H1 + n1, "PH");
    X.set("H2.aa", H2, "PPHH"); X.set("H2.ab", H2 + n4, "PPHH"); X.set("H2.bb", H2 + 2 * n4, "PPHH");
    X.use_id = 0;
    const Use ua = rename_use(C0, "T1", "U1", "T2", "U2"), ub = rename_use(C0, "E1", "H1", "E2", "H2");
    std::map<std::string, TensorRef> none_a, none_b;
    if (X.run_fused({&ua, &ub}, {&none_a, &none_b}, {energies + 1, energies + 2})) {
      relax_stage();
      mark(ev, 6, st);
      bo.W1 = W1; bo.W2 = W2; bo.Z1 = Z1; bo.Z2 = Z2; bo.U1 = U1; bo.U2 = U2;
      return bo;
    }
  }
  X.set("T1.a", U1, "PH"); X.set("T1.b", U1 + n1, "PH");
  X.set("T2.aa", U2, "PPHH", 1); X.set("T2.ab", U2 + n4, "PPHH"); X.set("T2.bb", U2 + 2 * n4, "PPHH", 1);
  scalar(energies + 1);
  // core-pair matrix P2[i][j] of E(3): gradient of each scalar with respect to its doubles
  // amplitudes on the core-core block, dotted with those amplitudes
  std::map<std::string, TensorRef> gout;
  double *G2 = nullptr, *P2 = nullptr;
  auto pair_part = [&](const double* Taa, const double* Tab, const double* Tbb) {
    op([G2, n4](hipStream_t s) { launch_fill(G2, 3 * (long long)n4, 0.0, s); });
    X.run_use(pair_use(), gout, nullptr);
    op([ad, G2, Taa, Tab, Tbb, P2](hipStream_t s) { launch_pair_dot(ad, G2, Taa, Tab, Tbb, P2, s); });
  };
  if (want_pairs) {
    G2 = pool.alloc(3 * n4);
    P2 = pool.alloc((size_t)std::max(1, nC * nC));
    const long long np2 = (long long)nC * nC;
    op([P2, np2](hipStream_t s) { launch_fill(P2, np2, 0.0, s); });
    auto mk = [&](double* p) {
      TensorRef t{p, "PPHH", {(long long)nP * nH * nH, (long long)nH * nH, nH, 1}, (long long)n4};
      return t;
    };
    gout["G2.aa"] = mk(G2);
    gout["G2.ab"] = mk(G2 + n4);
    gout["G2.bb"] = mk(G2 + 2 * n4);
    X.use_id = 3;
    pair_part(U2, U2 + n4, U2 + 2 * n4);
  }
  // E(3)_b = <[H~(2)_{1,2}, T(1)]>
  bind_first();
  if (rest) {
    // the rest of E(3)_b: first-order doubles without their core-core hole pairs
    double* Tm = pool.alloc(2 * n4);
    op([=](hipStream_t s) {
      launch_mask_core_pairs(ad, T2aa, Tm, 1, s);
      launch_mask_core_pairs(ad, T2ab, Tm + n4, 1, s);
    });
    X.set("T2.aa", Tm, "PPHH", 1); X.set("T2.ab", Tm + n4, "PPHH", 2); X.set("T2.bb", Tm, "PPHH", 1);
  }
  X.set("E1.a", H1, "PH"); X.set("E1.b", H1 + n1, "PH");
  X.set("E2.aa", H2, "PPHH"); X.set("E2.ab", H2 + n4, "PPHH"); X.set("E2.bb", H2 + 2 * n4, "PPHH");
  scalar(energies + 2);
  if (want_pairs) {
    X.use_id = 4;
    pair_part(T2aa, T2ab, T2aa);
    bo.pairs = pool.alloc((size_t)nC * (nC + 1) / 2 + 1);
    double* pairs = bo.pairs;
    op([nC, P2, energies, pairs](hipStream_t s) { launch_pair_fold(nC, P2, energies, pairs, s); });
  }
  relax_stage();
  mark(ev, 6, st);
  bo.W1 = W1; bo.W2 = W2; bo.Z1 = Z1; bo.Z2 = Z2; bo.U1 = U1; bo.U2 = U2;
  return bo;
}

// ---------------------------------------------------------------------------
// Plans: the pipeline of one shape, recorded while it first runs and captured into a HIP
// graph; later calls of the same shape copy their inputs and launch the graph.
// ---------------------------------------------------------------------------
struct Plan {
  std::string key;
  int device = 0;
  std::unique_ptr<Pool> pool;
  Inputs in;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double* pinned = nullptr;   // host [16]: s at [0], energies at [4..8), non-finite count at [8]
  bool busy = false;
  unsigned long long stamp = 0;
  double gett_flops = 0, ladder_flops = 0;
  int ladder_batch = 0, n_launch = 0, grouped_uses = 0, precision = 0;
  ~Plan() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    if (pinned) (void)hipHostFree(pinned);
    pool.reset();
    (void)hipSetDevice(cur);
  }
};

constexpr int kMaxPlans = 4;
constexpr size_t kMaxPlanBytes = 16ULL << 30;
static std::mutex g_plan_mu;
// never destroyed: freeing device memory during static destruction can outlive the runtime
static std::vector<std::unique_ptr<Plan>>& plans() {
  static auto* v = new std::vector<std::unique_ptr<Plan>>();
  return *v;
}
static unsigned long long g_plan_clock = 0;

static void capture(Plan& pl, std::vector<DevOp>& ops) {
  HIPCHECK(hipStreamCreateWithFlags(&pl.cap, hipStreamNonBlocking));
  HIPCHECK(hipStreamBeginCapture(pl.cap, hipStreamCaptureModeRelaxed));
  hipGraph_t g = nullptr;
  try {
    for (auto& f : ops) f(pl.cap);
    HIPCHECK(hipGetLastError());
  } catch (...) {
    if (hipStreamEndCapture(pl.cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    throw;
  }
  HIPCHECK(hipStreamEndCapture(pl.cap, &g));
  pl.graph = g;
  HIPCHECK(hipGraphInstantiate(&pl.exec, pl.graph, nullptr, nullptr, 0));
}

// Insert a new plan, dropping the least recently used idle plans beyond the limits.
static bool keep_plan(std::unique_ptr<Plan> fresh) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto& v = plans();
  v.push_back(std::move(fresh));
  auto over = [&] {
    size_t bytes = 0;
    for (auto& p : v) bytes += p->pool->bytes;
    return (int)v.size() > kMaxPlans || bytes > kMaxPlanBytes;
  };
  while (over()) {
    int victim = -1;
    for (int i = 0; i + 1 < (int)v.size(); ++i)
      if (!v[i]->busy && (victim < 0 || v[i]->stamp < v[victim]->stamp)) victim = i;
    if (victim < 0) {
      v.pop_back();   // the new plan (idle) does not fit beside busy ones
      return false;
    }
    v.erase(v.begin() + victim);
  }
  return true;
}

static void fill_result(dsrg_result* R, const double* e, bool pt3, double e0) {
  R->e2 = e[0];
  R->e3_a = pt3 ? e[1] : 0.0;
  R->e3_b = pt3 ? e[2] : 0.0;
  R->e3 = R->e3_a + R->e3_b;
  R->e_total = e0 + R->e2 + R->e3;   // Eq. E_unrelaxed
}

// Host-side checks of the densities (device inputs are checked on their device copies).
static void check_rdm_host(int nA, const double* g1, const double* g2) {
  const long long n2 = (long long)nA * nA, total = 2 * n2 + 3 * n2 * n2;
  for (long long e = 0; e < total; ++e)
    if (rdm_violations(nA, g1, g2, e))
      throw Error(DSRG_E_RDM, "gamma1 not symmetric or gamma2 not Hermitian/antisymmetric");
}

// s = +INFINITY (R_s = 1/D): every non-internal singles and doubles denominator must be
// away from zero.  Doubles: the pair sums e_i + e_j over holes and e_a + e_b over particles
// are sorted and the closest pair found by a merge (internal quadruples, all four active,
// carry no amplitude and are skipped by an exact scan of the active sums).
static void check_intruder(int nC, int nA, int nV, const double* eps) {
  const int nH = nC + nA, nP = nA + nV;
  const double tol = 1e-12;
  for (int i = 0; i < nH; ++i)
    for (int a = 0; a < nP; ++a) {
      if (i >= nC && a < nA) continue;   // internal
      if (std::fabs(eps[i] - eps[nC + a]) < tol)
        throw Error(DSRG_E_INTRUDER, "s = inf with a vanishing singles denominator");
    }
  // pairs touching at least one non-active index on either side
  struct PS { double v; bool all_active; };
  std::vector<PS> h, p;
  for (int i = 0; i < nH; ++i)
    for (int j = 0; j < nH; ++j) h.push_back({eps[i] + eps[j], i >= nC && j >= nC});
  for (int a = 0; a < nP; ++a)
    for (int b = 0; b < nP; ++b) p.push_back({eps[nC + a] + eps[nC + b], a < nA && b < nA});
  auto by = [](const PS& x, const PS& y) { return x.v < y.v; };
  std::sort(h.begin(), h.end(), by);
  std::sort(p.begin(), p.end(), by);
  // for every hole pair, the particle pairs within tol of it (two pointers)
  size_t lo = 0;
  for (const PS& x : h) {
    while (lo < p.size() && p[lo].v < x.v - tol) ++lo;
    for (size_t k = lo; k < p.size() && p[k].v <= x.v + tol; ++k)
      if (!(x.all_active && p[k].all_active) && std::fabs(x.v - p[k].v) < tol)
        throw Error(DSRG_E_INTRUDER, "s = inf with a vanishing doubles denominator");
  }
}

// Checked arguments of a call and the key of its plan.  slot > 0 keys a separate plan of
// the same shape (concurrent members of a batch).
// Tile rules by problem size (dsrg_set_tile_rules): the first rule whose particle-space
// range holds n_active + n_virtual applies to a call.
static std::mutex g_rules_mu;
static std::vector<dsrg_tile_rule> g_rules;

static dsrg_tile_rule rule_for(int nP) {
  std::lock_guard<std::mutex> lk(g_rules_mu);
  for (const auto& r : g_rules)
    if (nP >= r.np_min && nP <= r.np_max) return r;
  dsrg_tile_rule none;
  memset(&none, 0, sizeof(none));
  return none;
}

struct Setup {
  Shape sh;
  int prec = 0;   // DSRG_PRECISION_* of the contractions
  bool devptr = false, profile = false, grouped = true, unique_ladder = true;
  bool want_pairs = false, cacheable = false;
  long long cap = 0;
  long long group_cap = 0;   // bytes of temporaries one grouped commutator may hold
  int vb = 0;   // requested (PP|PP) batch (0: largest that fits)
  hipStream_t st = nullptr;
  int dev = 0;
  std::string key;
};

static Setup setup(const dsrg_problem* P, const dsrg_options* O, const dsrg_intermediates* I, bool pt3,
                   double* e3_pairs, double* e3_rest, int slot) {
  if (!P) throw Error(DSRG_E_ARG, "null problem or result");
  const int nC = P->n_core, nA = P->n_active, nV = P->n_virtual, M = P->n_aux;
  if (nC < 0 || nA < 0 || nV < 0) throw Error(DSRG_E_ARG, "negative orbital count");
  if (M < 1) throw Error(DSRG_E_ARG, "n_aux must be >= 1");
  if (nC + nA + nV < 1) throw Error(DSRG_E_ARG, "no orbitals");
  if (!(P->s > 0.0)) throw Error(DSRG_E_ARG, "s must be > 0");
  if (!P->eps || !P->B) throw Error(DSRG_E_ARG, "null eps or B");
  if (nA > 0 && (!P->gamma1 || !P->gamma2)) throw Error(DSRG_E_ARG, "null gamma1/gamma2 with nA > 0");
  if (nA > 16) throw Error(DSRG_E_UNSUPPORTED, "active spaces above 16 orbitals are not built");
  if (O && O->precision != DSRG_PRECISION_FP64 && O->precision != DSRG_PRECISION_FP32 &&
      O->precision != DSRG_PRECISION_BF16X3)
    throw Error(DSRG_E_UNSUPPORTED, "unknown precision");
  if (O && O->virt_batch < 0) throw Error(DSRG_E_ARG, "virt_batch must be >= 0");
  Setup S;
  S.vb = O ? O->virt_batch : 0;
  // the size class's tile rule: the large-tile threshold of this thread's launches and,
  // unless the options name one, the (PP|PP) batch
  const dsrg_tile_rule rule = rule_for(nA + nV);
  set_big_tile_min(rule.big_tile_min);
  if (S.vb == 0 && rule.virt_batch > 0) S.vb = rule.virt_batch;
  S.prec = O ? O->precision : DSRG_PRECISION_FP64;
  const int flags = O ? O->flags : 0;
  S.devptr = flags & DSRG_F_DEVICE_PTRS;
  S.profile = flags & DSRG_F_PROFILE;
  Shape& sh = S.sh;
  sh.nC = nC; sh.nA = nA; sh.nV = nV; sh.M = M;
  sh.N = nC + nA + nV;
  sh.nB = (long long)M * sh.N * sh.N;
  sh.g1n = 2LL * nA * nA;
  sh.g2n = 3LL * nA * nA * nA * nA;
  sh.g3n = 4LL * nA * nA * nA * nA * nA * nA;
  sh.has_g3 = nA > 0 && P->gamma3;
  sh.has_f = P->f_offdiag != nullptr;
  sh.pt3 = pt3;
  if (!S.devptr) {
    if (!finite_host(P->eps, sh.N) || !finite_host(P->B, sh.nB) ||
        (nA > 0 && (!finite_host(P->gamma1, sh.g1n) || !finite_host(P->gamma2, sh.g2n))) ||
        (sh.has_g3 && !finite_host(P->gamma3, sh.g3n)) ||
        (sh.has_f && !finite_host(P->f_offdiag, (size_t)(sh.N * sh.N))))
      throw Error(DSRG_E_NONFINITE, "non-finite value in eps, B, f_offdiag or the densities");
    if (nA > 0) check_rdm_host(nA, P->gamma1, P->gamma2);
  }
  if (std::isinf(P->s)) {
    // the unregularised limit: denominators checked on the host (eps copied if on the device)
    std::vector<double> e(sh.N);
    if (S.devptr) HIPCHECK(hipMemcpy(e.data(), P->eps, sh.N * sizeof(double), hipMemcpyDeviceToHost));
    else std::copy(P->eps, P->eps + sh.N, e.begin());
    for (double x : e)
      if (!std::isfinite(x)) throw Error(DSRG_E_NONFINITE, "non-finite value in eps");
    check_intruder(nC, nA, nV, e.data());
  }
  S.st = (O && O->stream) ? (hipStream_t)O->stream : (hipStream_t)0;
  S.cap = (O && O->workspace_cap > 0) ? O->workspace_cap : (48LL << 30);
  S.group_cap = (O && O->workspace_cap > 0) ? O->workspace_cap / 2 : (4LL << 30);
  S.grouped = !(flags & DSRG_F_NO_GROUPING);
  S.unique_ladder = !(flags & DSRG_F_FULL_LADDER);
  if (pt3 && nC + nA > 0 && nA + nV > 0) {
    // one value of the batch letter of the (PP|PP) ladder: nP^3 integrals plus, on unique
    // pairs, its antisymmetrised and symmetrised pair rows (the executor checks the same)
    const long long nP = nA + nV, kp = nP * (nP - 1) / 2;
    const long long row = 8 * (nP * nP * nP + (S.unique_ladder ? nP * (2 * kp + nP) : 0));
    if (S.cap < row)
      throw Error(DSRG_E_OOM, "workspace_cap of " + std::to_string(S.cap) + " bytes is below one (PP|PP) batch row of " +
                                  std::to_string(row) + " bytes");
    if (S.vb > 0 && (long long)std::min<long long>(S.vb, nP) * row > S.cap)
      throw Error(DSRG_E_OOM, "virt_batch " + std::to_string(S.vb) + " does not fit workspace_cap");
  }
  S.want_pairs = e3_rest != nullptr;
  if (S.want_pairs && nC > 0 && !e3_pairs) throw Error(DSRG_E_ARG, "null e3_pairs with n_core > 0");
  S.cacheable = !S.profile && !I && !S.want_pairs && !(flags & DSRG_F_NO_PLAN_CACHE);
  HIPCHECK(hipGetDevice(&S.dev));
  char kbuf[224];
  snprintf(kbuf, sizeof(kbuf), "%d:%d:%d:%d:%d:%d:%d:%d:%d:%d:%d:%lld:%d:%d:%d", S.dev, nC, nA, nV, M, (int)sh.has_g3,
           (int)sh.has_f, (int)pt3, (int)S.grouped, (int)S.unique_ladder, S.prec, S.cap, S.vb, slot,
           big_tile_min());
  S.key = kbuf;
  return S;
}

// An idle cached plan of this key, marked busy (null if there is none); seen tells whether
// one exists at all.
static Plan* acquire_plan(const std::string& key, bool& seen) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  seen = false;
  for (auto& p : plans())
    if (p->key == key) {
      seen = true;
      if (!p->busy) {
        p->busy = true;
        p->stamp = ++g_plan_clock;
        return p.get();
      }
    }
  return nullptr;
}

static void release_plan(Plan* p) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  p->busy = false;
}

// Library streams for the concurrent members of a batch (per device, default priority,
// created on first use and kept for the process).
constexpr int kBatchStreams = 4;   // streams created; a round uses batch_round() of them
// Members per round: every replay keeps two streams busy (its main sequence and the ladder
// beside it), so a round holds half the hardware queues HIP gives the process
// (GPU_MAX_HW_QUEUES, 4 unless set): more streams than queues share queues and serialise.
static int batch_round() {
  const char* q = getenv("GPU_MAX_HW_QUEUES");
  const int hwq = q ? atoi(q) : 4;
  return std::max(1, std::min(kBatchStreams, hwq / 2));
}
static hipStream_t* batch_streams(int dev) {
  static std::mutex mu;
  static std::map<int, std::vector<hipStream_t>> m;
  std::lock_guard<std::mutex> lk(mu);
  auto& v = m[dev];
  if (v.empty()) {
    v.assign(kBatchStreams, nullptr);
    for (auto& x : v)
      if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        for (auto& y : v)
          if (y) (void)hipStreamDestroy(y);
        v.clear();
        return nullptr;
      }
  }
  return v.data();
}

// Launches the replay of a cached plan on S.st without waiting: inputs (s read from s_src,
// non-finite count to bad for device inputs), the graph, the energies to e_dst (host,
// pinned).  The host buffers must stay untouched until the stream has passed the launch.
static void replay_launch(Plan* plan, const dsrg_problem* P, const Setup& S, const double* s_src,
                          double* e_dst, int* bad) {
  bad[0] = bad[1] = 0;
  load_inputs(P, S.devptr, S.sh, plan->in, s_src, S.st, S.devptr ? bad : nullptr);
  HIPCHECK(hipGraphLaunch(plan->exec, S.st));
  HIPCHECK(hipMemcpyAsync(e_dst, plan->in.energies, 4 * sizeof(double), hipMemcpyDeviceToHost, S.st));
}

static void replay_result(const Plan* plan, const double* e, bool pt3, double e0, dsrg_result* R) {
  dsrg_result r;
  memset(&r, 0, sizeof(r));
  fill_result(&r, e, pt3, e0);
  r.gett_flops = plan->gett_flops;
  r.ladder_flops = plan->ladder_flops;
  r.ladder_batch = plan->ladder_batch;
  r.n_launch = plan->n_launch;
  r.grouped_uses = plan->grouped_uses;
  r.plan = 2;
  r.alg_flops = plan->gett_flops;
  r.precision_used = plan->precision;
  r.virt_batch_used = plan->ladder_batch;
  *R = r;
}

// feat_host / e2p_host (both or neither): the rest-only mode (RestMode) with the core-pair
// features and second-order pair proxies copied to these host arrays
// One-step relaxation request: the CAS determinant space and what to copy back.
struct RelaxReq {
  int n_alpha = 0, n_beta = 0;
  const double* ci_guess = nullptr;
  bool want_ci = false, want_blocks = false;
  dsrg_cas::Out out;
};

static int run(const dsrg_problem* P, const dsrg_options* O, dsrg_result* R,
               const dsrg_intermediates* I, bool pt3, double* e3_pairs = nullptr,
               double* e3_rest = nullptr, int slot = 0, float* feat_host = nullptr,
               double* e2p_host = nullptr, RelaxReq* rq = nullptr) {
  if (!P || !R) throw Error(DSRG_E_ARG, "null problem or result");
  Setup S = setup(P, O, I, pt3, e3_pairs, e3_rest, slot);
  const bool rest_mode = feat_host != nullptr;
  if (rest_mode || rq) S.cacheable = false;
  const Shape& sh = S.sh;
  const int nC = sh.nC, nA = sh.nA, nV = sh.nV, M = sh.M;
  const int prec = S.prec;
  const bool devptr = S.devptr, profile = S.profile, grouped = S.grouped;
  const bool unique_ladder = S.unique_ladder, want_pairs = S.want_pairs, cacheable = S.cacheable;
  hipStream_t st = S.st;
  const long long cap = S.cap;
  const int dev = S.dev;
  const std::string& key = S.key;
  Plan* plan = nullptr;
  std::unique_ptr<Plan> fresh;
  if (cacheable) {
    bool seen = false;
    plan = acquire_plan(key, seen);
    // a plan of this shape in use by another thread: run without one
    if (!seen) {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      fresh = std::make_unique<Plan>();
      fresh->key = key;
      fresh->device = dev;
      fresh->stamp = ++g_plan_clock;
    }
  }

  hipEvent_t ev[8];
  for (auto& e : ev) HIPCHECK(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 8; ++i) (void)hipEventDestroy(e[i]); }
  } evg{ev};
  dsrg_result r;
  memset(&r, 0, sizeof(r));

  if (plan) {
    struct Release {
      Plan* p;
      ~Release() { release_plan(p); }
    } rel{plan};
    plan->pinned[0] = P->s;
    // device inputs: the non-finite check runs ahead of the graph and is read after it
    int* bad = reinterpret_cast<int*>(plan->pinned + 8);
    bad[0] = bad[1] = 0;
    load_inputs(P, devptr, sh, plan->in, plan->pinned, st, devptr ? bad : nullptr);
    mark(ev, 0, st);
    HIPCHECK(hipGraphLaunch(plan->exec, st));
    mark(ev, 7, st);
    HIPCHECK(hipMemcpyAsync(plan->pinned + 4, plan->in.energies, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    check_bad(bad);
    fill_result(&r, plan->pinned + 4, pt3, P->e0);
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, ev[0], ev[7]));
    r.t_seconds[7] = ms * 1e-3;
    r.gett_flops = plan->gett_flops;
    r.ladder_flops = plan->ladder_flops;
    r.ladder_batch = plan->ladder_batch;
    r.n_launch = plan->n_launch;
    r.grouped_uses = plan->grouped_uses;
    r.plan = 2;
    r.alg_flops = plan->gett_flops;
    r.precision_used = plan->precision;
    r.virt_batch_used = plan->ladder_batch;
    *R = r;
    return DSRG_OK;
  }

  std::unique_ptr<Pool> local;
  Pool* pool;
  const double* s_src = &P->s;   // lives until the synchronisation below
  if (fresh) {
    fresh->pool = std::make_unique<Pool>(st, true);
    pool = fresh->pool.get();
    HIPCHECK(hipHostMalloc((void**)&fresh->pinned, 16 * sizeof(double), hipHostMallocDefault));
    fresh->pinned[0] = P->s;
    s_src = fresh->pinned;
  } else {
    local = std::make_unique<Pool>(st);
    pool = local.get();
  }
  Inputs in = alloc_inputs(*pool, sh);
  load_inputs(P, devptr, sh, in, s_src, st);
  std::vector<DevOp> ops;
  OpLog op{st, fresh ? &ops : nullptr};
  Exec X(Dims{nC, nA, nV}, st, *pool, op, in.B, M, cap, profile);
  X.grouped = grouped;
  X.unique_ladder = unique_ladder;
  X.group_cap = S.group_cap;
  X.prec = prec;
  X.virt_batch = S.vb;
  mark(ev, 0, st);
  RestOut ro;
  BodyOut bo = body(X, op, *pool, sh, in, ev, st, want_pairs, rest_mode ? &ro : nullptr, rq != nullptr);
  if (rest_mode && nC > 0) {
    const size_t np = (size_t)nC * (nC + 1) / 2;
    HIPCHECK(hipMemcpyAsync(feat_host, ro.feat, np * 16 * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(e2p_host, ro.e2, np * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  std::vector<double> pair_host;
  if (want_pairs) {
    const size_t np = (size_t)nC * (nC + 1) / 2 + 1;
    pair_host.resize(np);
    HIPCHECK(hipMemcpyAsync(pair_host.data(), bo.pairs, np * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (I) {
    const size_t nH = nC + nA, nP = nA + nV, n1 = nP * nH, n4 = nP * nP * nH * nH;
    auto cp = [&](double* h, const double* dptr, size_t n) {
      if (h && dptr) HIPCHECK(hipMemcpyAsync(h, dptr, n * 8, hipMemcpyDeviceToHost, st));
    };
    cp(I->t1, bo.T1a, n1);
    cp(I->t1 ? I->t1 + n1 : nullptr, bo.T1b, n1);
    cp(I->t2, bo.T2aa, n4);
    cp(I->t2 ? I->t2 + n4 : nullptr, bo.T2ab, n4);
    cp(I->t2 ? I->t2 + 2 * n4 : nullptr, bo.T2aa, n4);
    cp(I->w1, bo.W1, 2 * n1); cp(I->w2, bo.W2, 3 * n4);
    cp(I->z1, bo.Z1, 2 * n1); cp(I->z2, bo.Z2, 3 * n4);
    cp(I->u1, bo.U1, 2 * n1); cp(I->u2, bo.U2, 3 * n4);
  }
  mark(ev, 7, st);
  double e[4] = {0, 0, 0, 0};
  HIPCHECK(hipMemcpyAsync(e, in.energies, 4 * 8, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  HIPCHECK(hipGetLastError());
  fill_result(&r, e, pt3, P->e0);
  float ms;
  for (int k = 0; k < 6; ++k) {
    HIPCHECK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
    r.t_seconds[k] = ms * 1e-3;
  }
  HIPCHECK(hipEventElapsedTime(&ms, ev[0], ev[7]));
  r.t_seconds[7] = ms * 1e-3;
  if (X.profile) X.collect_profile();
  for (int k = 0; k < kRoles; ++k) {
    r.role_seconds[k] = X.role_sec[k];
    r.role_flops[k] = X.role_flops[k];
    r.role_bytes[k] = X.role_bytes[k];
    r.role_launches[k] = X.role_n[k];
  }
  for (int k = 0; k < 2 * kRoles; ++k) {
    r.kernel_seconds[k] = X.kern_sec[k];
    r.kernel_flops[k] = X.kern_flops[k];
    r.kernel_launches[k] = X.kern_n[k];
  }
  r.gett_flops = X.gett_flops;
  r.ladder_flops = X.ladder_flops;
  r.ladder_seconds = X.ladder_ms * 1e-3;
  r.ladder_batch = X.ladder_batch;
  r.n_launch = X.n_launch;
  r.grouped_uses = X.grouped_uses;
  r.alg_flops = X.gett_flops;
  r.precision_used = prec;
  r.virt_batch_used = X.ladder_batch;
  *R = r;
  if (want_pairs) {
    const size_t np = (size_t)nC * (nC + 1) / 2;
    if (np) memcpy(e3_pairs, pair_host.data(), np * sizeof(double));
    *e3_rest = pair_host[np];
  }
  if (rq) {
    // the CAS eigenproblem of Hbar^[3]_{1,2} after the pipeline (its own host-driven loop)
    dsrg_cas::In ci;
    ci.nC = nC; ci.nA = nA; ci.nV = nV; ci.M = M;
    ci.eps = in.eps; ci.B = in.B; ci.g1 = in.g1; ci.g2 = in.g2; ci.energies = in.energies; ci.R = bo.R;
    ci.n_alpha = rq->n_alpha; ci.n_beta = rq->n_beta; ci.ci_guess = rq->ci_guess;
    try {
      dsrg_cas::relax(ci, st, rq->want_ci, rq->want_blocks, rq->out);
    } catch (const dsrg_cas::Err& e) {
      throw Error(e.code, e.what());
    }
  }

  if (fresh && pool->bytes <= kMaxPlanBytes) {
    // capture the recorded pipeline; a failure only means later calls run without a plan
    fresh->in = in;
    fresh->gett_flops = X.gett_flops;
    fresh->ladder_flops = X.ladder_flops;
    fresh->ladder_batch = X.ladder_batch;
    fresh->n_launch = X.n_launch;
    fresh->grouped_uses = X.grouped_uses;
    fresh->precision = r.precision_used;
    try {
      capture(*fresh, ops);
      // from here on every use of the plan ends with a synchronisation of its caller's stream
      fresh->pool->sync_before_free = false;
      if (keep_plan(std::move(fresh))) R->plan = 1;
    } catch (const Error&) {
      (void)hipGetLastError();
    }
  }
  return DSRG_OK;
}

// the pair-energy network's entry points report errors through the same message
void set_last_error(const char* m) { g_last_error = m; }

template <class F>
static int guarded(F&& f) {
  try {
    int rc = f();
    g_last_error.clear();
    return rc;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return DSRG_E_HIP;
  }
}

// ---------------------------------------------------------------------------
// Allocation-free entry: every buffer of the pipeline carved from a static device array.
// The pipeline is planned first with its launches recorded but not run, so a problem that
// does not fit fails before any device work; then the inputs are copied and the recorded
// launches run in order on the caller's stream.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)DSRG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

struct ScratchDev {
  char* ptr = nullptr;   // this device's copy of the array (device address)
  std::mutex call;       // calls on one device share the array: one at a time
};
// Set up on the first call on a device (that device current): the array's device address
// from the runtime, kept per device.  The host-side name of the array is never used as an
// address.
static ScratchDev& scratch_dev(int dev) {
  static std::mutex mu;
  static auto* m = new std::map<int, std::unique_ptr<ScratchDev>>();
  std::lock_guard<std::mutex> lk(mu);
  auto& e = (*m)[dev];
  if (!e) {
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(DSRG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc));
    }
    auto d = std::make_unique<ScratchDev>();
    d->ptr = static_cast<char*>(p);
    e = std::move(d);
  }
  return *e;
}

static int run_noalloc(const dsrg_problem* P, const dsrg_options* O, dsrg_result* R) {
  if (!P || !R) throw Error(DSRG_E_ARG, "null problem or result");
  if (O && (O->flags & DSRG_F_PROFILE)) throw Error(DSRG_E_ARG, "DSRG_F_PROFILE needs events: not available without allocation");
  const Setup S = setup(P, O, nullptr, true, nullptr, nullptr, 0);
  const Shape& sh = S.sh;
  ScratchDev& sd = scratch_dev(S.dev);
  std::lock_guard<std::mutex> lk(sd.call);
  Pool pool(S.st, sd.ptr, kScratchBytes);
  Inputs in = alloc_inputs(pool, sh);
  std::vector<DevOp> ops;
  OpLog op{S.st, &ops};
  op.defer = true;
  // the (PP|PP) batches and the grouped temporaries get at most a quarter of the array
  const long long cap = std::min<long long>(S.cap, (long long)(kScratchBytes / 4));
  Exec X(Dims{sh.nC, sh.nA, sh.nV}, S.st, pool, op, in.B, sh.M, cap, false);
  X.grouped = S.grouped;
  X.unique_ladder = S.unique_ladder;
  X.group_cap = cap / 2;
  X.prec = S.prec;
  X.virt_batch = S.vb;
  X.no_side = true;
  body(X, op, pool, sh, in, nullptr, S.st, false);   // plans and records every launch
  load_inputs(P, S.devptr, sh, in, &P->s, S.st);
  for (auto& f : ops) f(S.st);
  double e[4] = {0, 0, 0, 0};
  HIPCHECK(hipMemcpyAsync(e, in.energies, 4 * sizeof(double), hipMemcpyDeviceToHost, S.st));
  HIPCHECK(hipStreamSynchronize(S.st));
  HIPCHECK(hipGetLastError());
  dsrg_result r;
  memset(&r, 0, sizeof(r));
  fill_result(&r, e, true, P->e0);
  r.gett_flops = X.gett_flops;
  r.ladder_flops = X.ladder_flops;
  r.ladder_batch = X.ladder_batch;
  r.n_launch = X.n_launch;
  r.grouped_uses = X.grouped_uses;
  r.alg_flops = X.gett_flops;
  r.precision_used = S.prec;
  r.virt_batch_used = X.ladder_batch;
  *R = r;
  return DSRG_OK;
}

}  // namespace dsrg

extern "C" {

int dsrg_pt2_energy(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out) {
  return dsrg::guarded([&] { return dsrg::run(prob, opt, out, nullptr, false); });
}

int dsrg_pt3_energy(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out) {
  return dsrg::guarded([&] { return dsrg::run(prob, opt, out, nullptr, true); });
}

int dsrg_pt3_energy_batch(const dsrg_problem* probs, int32_t n, const dsrg_options* opt,
                          dsrg_result* outs, int32_t* status) {
  if (!probs || !outs || !status || n < 1) {
    dsrg::g_last_error = "null arrays or n < 1";
    return DSRG_E_ARG;
  }
  // Members run in rounds of K = batch_round(): member k on library stream k % K
  // (ordered after the caller's stream) with a plan of its own slot, so the members of a
  // round overlap on the GPU.  Each member's s, energies and non-finite count go through its
  // own pinned slot.  Members without a cached plan (a shape not seen before) run their
  // pipeline directly and record a plan: small ones on worker threads, one per stream of
  // the round, large ones alone on the calling thread.
  int dev = 0;
  hipStream_t caller = (opt && opt->stream) ? (hipStream_t)opt->stream : (hipStream_t)0;
  hipStream_t* ss = nullptr;
  hipEvent_t ready = nullptr;
  double* stage = nullptr;   // per member: s, 4 energies, non-finite count
  constexpr int kStage = 8;
  if (hipGetDevice(&dev) != hipSuccess || !(ss = dsrg::batch_streams(dev)) ||
      hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&stage, (size_t)n * kStage * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    // no streams or staging (e.g. no device): the members one call after another, each
    // with its own checks and error
    (void)hipGetLastError();
    if (ready) (void)hipEventDestroy(ready);
    int first_error = DSRG_OK;
    bool any_ok = false;
    for (int32_t k = 0; k < n; ++k) {
      status[k] = dsrg::guarded([&] { return dsrg::run(probs + k, opt, outs + k, nullptr, true); });
      if (status[k] == DSRG_OK) any_ok = true;
      else if (first_error == DSRG_OK) first_error = status[k];
    }
    return any_ok ? DSRG_OK : first_error;
  }
  const int K = std::min<int>(n, dsrg::batch_round());
  (void)hipEventRecord(ready, caller);
  for (int j = 0; j < K; ++j) (void)hipStreamWaitEvent(ss[j], ready, 0);
  std::map<std::string, dsrg::Plan*> held;   // plans this batch holds (busy) until its end
  std::vector<dsrg::Plan*> used(n, nullptr);
  std::vector<dsrg_options> oj(n);
  std::vector<std::string> werr(n);           // messages of members run on worker threads
  std::vector<char> pt3v(n, 1);
  for (int32_t r0 = 0; r0 < n; r0 += K) {
    // rounds of K members: more graphs in flight than the hardware queues serve (each
    // replay has a side branch) ran slower than two at a time
    if (r0 > 0)
      for (int i = 0; i < K; ++i) (void)hipStreamSynchronize(ss[i]);
    // members without a cached plan run their whole pipeline on worker threads, one per
    // library stream, so uneven shapes (a plan each) overlap on the GPU as replays do
    std::vector<std::thread> workers;
    for (int32_t k = r0; k < std::min<int32_t>(n, r0 + K); ++k) {
      const int j = k - r0;
      memset(&oj[k], 0, sizeof(dsrg_options));
      if (opt) oj[k] = *opt;
      oj[k].stream = ss[j];
      bool direct = false;
      status[k] = dsrg::guarded([&] {
        const dsrg::Setup S = dsrg::setup(probs + k, &oj[k], nullptr, true, nullptr, nullptr, j);
        dsrg::Plan* plan = nullptr;
        if (S.cacheable) {
          auto it = held.find(S.key);
          if (it != held.end()) {
            plan = it->second;
          } else {
            bool seen = false;
            plan = dsrg::acquire_plan(S.key, seen);
            if (plan) held[S.key] = plan;
          }
        }
        if (!plan) {
          direct = true;
          return DSRG_OK;
        }
        double* st_k = stage + (size_t)k * kStage;
        st_k[0] = probs[k].s;
        dsrg::replay_launch(plan, probs + k, S, st_k, st_k + 1, reinterpret_cast<int*>(st_k + 5));
        used[k] = plan;
        return DSRG_OK;
      });
      // a member too large to gain from sharing the GPU (its first-order doubles above 2^22
      // elements: two such members at once took longer than one after the other) runs
      // alone on this thread; smaller ones overlap on worker threads
      const long long nPm = (long long)probs[k].n_active + probs[k].n_virtual;
      const long long nHm = (long long)probs[k].n_core + probs[k].n_active;
      if (status[k] == DSRG_OK && direct && nPm * nPm * nHm * nHm > (1LL << 22)) {
        status[k] = dsrg::guarded([&] { return dsrg::run(probs + k, &oj[k], outs + k, nullptr, true, nullptr, nullptr, j); });
        if (status[k] != DSRG_OK) werr[k] = dsrg::g_last_error;
      } else if (status[k] == DSRG_OK && direct) {
        workers.emplace_back([&, k, j] {
          if (hipSetDevice(dev) != hipSuccess) {
            status[k] = DSRG_E_HIP;
            werr[k] = "hipSetDevice failed on a batch worker";
            return;
          }
          status[k] = dsrg::guarded([&] { return dsrg::run(probs + k, &oj[k], outs + k, nullptr, true, nullptr, nullptr, j); });
          if (status[k] != DSRG_OK) werr[k] = dsrg::g_last_error;
        });
      }
    }
    for (auto& w : workers) w.join();
  }
  int sync_rc = DSRG_OK;
  for (int j = 0; j < K; ++j)
    if (hipStreamSynchronize(ss[j]) != hipSuccess) sync_rc = DSRG_E_HIP;
  if (hipGetLastError() != hipSuccess) sync_rc = DSRG_E_HIP;
  int first_error = DSRG_OK;
  bool any_ok = false;
  for (int32_t k = 0; k < n; ++k) {
    if (status[k] == DSRG_OK && used[k]) {
      const double* st_k = stage + (size_t)k * kStage;
      if (sync_rc != DSRG_OK) status[k] = sync_rc;
      else if (reinterpret_cast<const int*>(st_k + 5)[0]) status[k] = DSRG_E_NONFINITE;
      else if (reinterpret_cast<const int*>(st_k + 5)[1]) status[k] = DSRG_E_RDM;
      else dsrg::replay_result(used[k], st_k + 1, pt3v[k], probs[k].e0, outs + k);
    }
    if (status[k] == DSRG_OK) any_ok = true;
    else if (first_error == DSRG_OK) first_error = status[k];
  }
  if (sync_rc != DSRG_OK) dsrg::g_last_error = "a batch stream failed";
  else
    for (int32_t k = 0; k < n; ++k)
      if (!werr[k].empty()) {
        dsrg::g_last_error = "member " + std::to_string(k) + ": " + werr[k];
        break;
      }
  for (auto& kv : held) dsrg::release_plan(kv.second);
  (void)hipHostFree(stage);
  (void)hipEventDestroy(ready);
  return any_ok ? DSRG_OK : first_error;
}

int dsrg_pair_features(const dsrg_problem* prob, const dsrg_options* opt, float* features, double* e2_pairs) {
  return dsrg::guarded([&] {
    if (!prob) throw dsrg::Error(DSRG_E_ARG, "null problem");
    if (prob->n_core > 0 && (!features || !e2_pairs)) throw dsrg::Error(DSRG_E_ARG, "null features or e2_pairs");
    float dummy_f[16];
    double dummy_e;
    dsrg_result r;
    return dsrg::run(prob, opt, &r, nullptr, false, nullptr, nullptr, 0, features ? features : dummy_f,
                     e2_pairs ? e2_pairs : &dummy_e);
  });
}

int dsrg_pt3_energy_surrogate(const dsrg_problem* prob, const dsrg_options* opt, const void* weights,
                              double rel_threshold, dsrg_result* out, int32_t* n_exact_pairs) {
  return dsrg::guarded([&] {
    if (!prob || !out || !weights) throw dsrg::Error(DSRG_E_ARG, "null problem, result or weights");
    if (!(rel_threshold >= 0.0)) throw dsrg::Error(DSRG_E_ARG, "rel_threshold must be >= 0");
    const int nC = prob->n_core;
    const size_t np = nC > 0 ? (size_t)nC * (nC + 1) / 2 : 0;
    std::vector<float> feat(std::max<size_t>(1, np) * 16);
    std::vector<double> e2p(std::max<size_t>(1, np)), pred(std::max<size_t>(1, np));
    dsrg_result r;
    dsrg::run(prob, opt, &r, nullptr, true, nullptr, nullptr, 0, feat.data(), e2p.data());
    // predicted core-pair parts: y = e3_ij / |E2_ij|^{3/2}, invariant under B -> kappa B
    int rc = np ? dsrg_mlp_predict(weights, feat.data(), (int64_t)np, pred.data()) : DSRG_OK;
    if (rc != DSRG_OK) throw dsrg::Error(rc, std::string("pair-energy network: ") + dsrg::g_last_error);
    std::vector<double> e3p(np);
    double mag = 0.0;
    for (size_t k = 0; k < np; ++k) {
      e3p[k] = pred[k] * std::pow(std::fabs(e2p[k]), 1.5);
      mag += std::fabs(e3p[k]);
    }
    // exact fallback: pairs predicted above rel_threshold of the summed magnitude, or whose
    // features lie far outside the training distribution (|z| > 8)
    const float* blob = static_cast<const float*>(weights);
    std::vector<char> exact(np, 0);
    int nexact = 0;
    for (size_t k = 0; k < np; ++k) {
      bool ood = false;
      for (int f = 0; f < 16; ++f)
        ood = ood || std::fabs((feat[k * 16 + f] - blob[8 + f]) / blob[24 + f]) > 8.0f;
      if (ood || std::fabs(e3p[k]) > rel_threshold * mag) {
        exact[k] = 1;
        ++nexact;
      }
    }
    if (nexact) {
      std::vector<double> pairs(np);
      double restv = 0;
      dsrg_result rf;
      dsrg::run(prob, opt, &rf, nullptr, true, pairs.data(), &restv);
      for (size_t k = 0; k < np; ++k)
        if (exact[k]) e3p[k] = pairs[k];
    }
    double sum = 0.0;
    for (size_t k = 0; k < np; ++k) sum += e3p[k];
    r.e3_b += sum;
    r.e3 = r.e3_a + r.e3_b;
    r.e_total = prob->e0 + r.e2 + r.e3;
    *out = r;
    if (n_exact_pairs) *n_exact_pairs = nexact;
    return DSRG_OK;
  });
}

int dsrg_pt3_energy_noalloc(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out) {
  return dsrg::guarded([&] { return dsrg::run_noalloc(prob, opt, out); });
}

int dsrg_pt3_pair_energies(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out,
                           double* e3_pairs, double* e3_rest) {
  return dsrg::guarded([&] {
    if (!e3_rest) throw dsrg::Error(DSRG_E_ARG, "null e3_rest");
    return dsrg::run(prob, opt, out, nullptr, true, e3_pairs, e3_rest);
  });
}

int dsrg_pt3_energy_ex(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out,
                       const dsrg_intermediates* inter) {
  return dsrg::guarded([&] { return dsrg::run(prob, opt, out, inter, true); });
}

int dsrg_set_tile_rules(const dsrg_tile_rule* rules, int32_t n) {
  if (n < 0 || (n > 0 && !rules)) {
    dsrg::g_last_error = "null rules or n < 0";
    return DSRG_E_ARG;
  }
  for (int32_t k = 0; k < n; ++k)
    if (rules[k].np_min > rules[k].np_max || rules[k].big_tile_min < 0 || rules[k].virt_batch < 0) {
      dsrg::g_last_error = "rule " + std::to_string(k) + ": np_min > np_max or a negative setting";
      return DSRG_E_ARG;
    }
  std::lock_guard<std::mutex> lk(dsrg::g_rules_mu);
  dsrg::g_rules.assign(rules, rules + n);
  dsrg::g_last_error.clear();
  return DSRG_OK;
}

int dsrg_dyall_aavv(const dsrg_problem* prob, const dsrg_options* opt, double* t_out, double* dmin) {
  return dsrg::guarded([&] {
    using namespace dsrg;
    if (!prob || !t_out) throw Error(DSRG_E_ARG, "null problem or t_out");
    if (prob->n_active == 0 || prob->n_active > dsrg_dyall::kMaxActive)
      throw Error(DSRG_E_UNSUPPORTED, "the Dyall active-to-virtual solve takes 1 to 9 active orbitals");
    const Setup S = setup(prob, opt, nullptr, false, nullptr, nullptr, 0);
    const Shape& sh = S.sh;
    const int nC = sh.nC, nA = sh.nA, nV = sh.nV;
    hipStream_t st = S.st;
    Pool pool(st);
    Inputs in = alloc_inputs(pool, sh);
    load_inputs(prob, S.devptr, sh, in, &prob->s, st);
    OpLog op{st, nullptr};
    Exec X(Dims{nC, nA, nV}, st, pool, op, in.B, sh.M, S.cap, false);
    double* Jvava = X.jblock("VAVA");   // [e][u][f][v] = (eu|fv)
    double* Jaaaa = X.jblock("AAAA");   // [x][u][y][v] = (xu|yv)
    const size_t np = (size_t)nA * (nA - 1) / 2, n2 = (size_t)nA * nA;
    double* Kaa = pool.alloc(np * np);
    double* Kbb = pool.alloc(np * np);
    double* Kab = pool.alloc(n2 * n2);
    const size_t nt = 3 * (size_t)nV * nV * n2;
    double* t = S.devptr ? t_out : pool.alloc(nt);
    const long long nsys = 3LL * nV * nV;
    double* dm = pool.alloc((size_t)std::max<long long>(nsys, 1) + 2);
    int* sing = reinterpret_cast<int*>(dm + std::max<long long>(nsys, 1) + 1);
    launch_fill(dm + std::max<long long>(nsys, 1), 2, 0.0, st);
    dsrg_dyall::launch_operator(nA, Jaaaa, in.g1, Kaa, Kbb, Kab, st);
    HIPCHECK(hipGetLastError());
    dsrg_dyall::launch_solve(nC, nA, nV, in.eps, Jvava, Kaa, Kbb, Kab, t, dm, sing, st);
    HIPCHECK(hipGetLastError());
    double* dres = dm + std::max<long long>(nsys, 1);   // the minimum over all blocks
    int hsing = 0;
    HIPCHECK(hipMemcpyAsync(&hsing, sing, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (hsing) throw Error(DSRG_E_INTRUDER, "a block of the active-to-virtual system is singular");
    if (nsys > 0) dsrg_dyall::launch_min(dm, nsys, dres, st);
    else launch_fill(dres, 1, INFINITY, st);
    HIPCHECK(hipGetLastError());
    double hmin = INFINITY;
    HIPCHECK(hipMemcpyAsync(&hmin, dres, sizeof(double), hipMemcpyDeviceToHost, st));
    if (!S.devptr) HIPCHECK(hipMemcpyAsync(t_out, t, nt * sizeof(double), hipMemcpyDeviceToHost, st));
    else if (dmin) HIPCHECK(hipMemcpyAsync(dmin, dres, sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    HIPCHECK(hipGetLastError());
    if (dmin && !S.devptr) *dmin = hmin;
    return DSRG_OK;
  });
}

int dsrg_pt3_energy_relaxed(const dsrg_problem* prob, int32_t n_alpha, int32_t n_beta, const double* ci_guess,
                            const dsrg_options* opt, dsrg_result* out, dsrg_relaxed_result* rel,
                            const dsrg_relaxed_outputs* outs) {
  return dsrg::guarded([&] {
    using dsrg::Error;
    if (!prob || !out || !rel) throw Error(DSRG_E_ARG, "null problem, result or relaxed result");
    const int nA = prob->n_active;
    if (nA < 0 || n_alpha < 0 || n_beta < 0 || n_alpha > nA || n_beta > nA)
      throw Error(DSRG_E_ARG, "n_alpha and n_beta must lie in [0, n_active]");
    auto binom = [](int n, int k) {
      long long r = 1;
      for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
      return r;
    };
    const long long ndet = binom(nA, n_alpha) * binom(nA, n_beta);
    // the determinant matrix is held densely: at most 2^27 elements (1 GiB)
    if (ndet > 11585) throw Error(DSRG_E_UNSUPPORTED, "CAS spaces above 11585 determinants are not built");
    if (nA > 0 && prob->gamma1) {
      std::vector<double> g((size_t)2 * nA * nA);
      if (opt && (opt->flags & DSRG_F_DEVICE_PTRS))
        HIPCHECK(hipMemcpy(g.data(), prob->gamma1, g.size() * sizeof(double), hipMemcpyDeviceToHost));
      else
        std::copy(prob->gamma1, prob->gamma1 + g.size(), g.begin());
      double ta = 0, tb = 0;
      for (int u = 0; u < nA; ++u) {
        ta += g[(size_t)u * nA + u];
        tb += g[(size_t)nA * nA + (size_t)u * nA + u];
      }
      // a non-finite gamma1 is left to the input checks of the pipeline
      if (std::isfinite(ta) && std::isfinite(tb) &&
          (std::fabs(ta - n_alpha) > 1e-8 || std::fabs(tb - n_beta) > 1e-8))
        throw Error(DSRG_E_RDM, "the traces of gamma1 differ from n_alpha, n_beta");
    }
    if (ci_guess && nA > 0 && !dsrg::finite_host(ci_guess, (size_t)ndet))
      throw Error(DSRG_E_NONFINITE, "non-finite value in ci_guess");
    dsrg::RelaxReq rq;
    rq.n_alpha = n_alpha;
    rq.n_beta = n_beta;
    rq.ci_guess = nA > 0 ? ci_guess : nullptr;
    rq.want_ci = outs && outs->ci;
    rq.want_blocks = outs && (outs->hbar1 || outs->hbar2 || outs->cas_c);
    dsrg_result r;
    const int rc = dsrg::run(prob, opt, &r, nullptr, true, nullptr, nullptr, 0, nullptr, nullptr, &rq);
    dsrg_relaxed_result x;
    memset(&x, 0, sizeof(x));
    x.e_relaxed = prob->e0 + rq.out.lambda;
    x.e_unrelaxed = r.e_total;
    x.cas_const = rq.out.cconst;
    x.residual = rq.out.residual;
    x.n_det = rq.out.n_det;
    x.iterations = rq.out.iterations;
    x.converged = rq.out.converged;
    if (outs) {
      if (outs->ci && !rq.out.ci.empty()) std::copy(rq.out.ci.begin(), rq.out.ci.end(), outs->ci);
      if (nA > 0) {
        if (outs->hbar1) std::copy(rq.out.h1.begin(), rq.out.h1.end(), outs->hbar1);
        if (outs->hbar2) std::copy(rq.out.h2.begin(), rq.out.h2.end(), outs->hbar2);
        if (outs->cas_c) std::copy(rq.out.c.begin(), rq.out.c.end(), outs->cas_c);
      }
    }
    *out = r;
    *rel = x;
    return rc;
  });
}

const char* dsrg_last_error(void) { return dsrg::g_last_error.c_str(); }

int dsrg_version(void) { return 100; }

int dsrg_release_cache(void) {
  return dsrg::guarded([&] {
    {
      std::lock_guard<std::mutex> lk(dsrg::g_plan_mu);
      auto& v = dsrg::plans();
      for (size_t i = v.size(); i-- > 0;)
        if (!v[i]->busy) v.erase(v.begin() + i);
    }
    dsrg::big_cache().clear();
    return DSRG_OK;
  });
}

}  // extern "C"

extern "C" int dsrg_test_gett(int nm, const int* md, const long long* am, const long long* cm,
                              int nn, const int* nd, const long long* bn, const long long* cn,
                              int nk, const int* kd, const long long* ak, const long long* bk,
                              const double* A, long long na, const double* B, long long nb,
                              double* C, long long nc, double alpha, int beta, int precision) {
  using namespace dsrg;
  return guarded([&] {
    if (nm < 0 || nn < 0 || nk < 0 || nm > kMaxComp || nn > kMaxComp || nk > kMaxComp)
      throw Error(DSRG_E_ARG, "component count out of range");
    if (!A || !B || !C || na <= 0 || nb <= 0 || nc <= 0) throw Error(DSRG_E_ARG, "null or empty array");
    if (precision != DSRG_PRECISION_FP64 && precision != DSRG_PRECISION_FP32 &&
        precision != DSRG_PRECISION_BF16X3)
      throw Error(DSRG_E_UNSUPPORTED, "unknown precision");
    GettDesc g;
    g.nm = nm; g.nn = nn; g.nk = nk;
    long long M = 1, N = 1, K = 1, amax = 0, bmax = 0, cmax = 0;
    for (int i = 0; i < nm; ++i) {
      if (md[i] < 1) throw Error(DSRG_E_ARG, "extent < 1");
      g.md[i] = md[i]; g.am[i] = am[i]; g.cm[i] = cm[i]; M *= md[i];
      amax += (md[i] - 1) * std::abs(am[i]); cmax += (md[i] - 1) * std::abs(cm[i]);
    }
    for (int i = 0; i < nn; ++i) {
      if (nd[i] < 1) throw Error(DSRG_E_ARG, "extent < 1");
      g.nd[i] = nd[i]; g.bn[i] = bn[i]; g.cn[i] = cn[i]; N *= nd[i];
      bmax += (nd[i] - 1) * std::abs(bn[i]); cmax += (nd[i] - 1) * std::abs(cn[i]);
    }
    for (int i = 0; i < nk; ++i) {
      if (kd[i] < 1) throw Error(DSRG_E_ARG, "extent < 1");
      g.kd[i] = kd[i]; g.ak[i] = ak[i]; g.bk[i] = bk[i]; K *= kd[i];
      amax += (kd[i] - 1) * std::abs(ak[i]); bmax += (kd[i] - 1) * std::abs(bk[i]);
    }
    for (int i = 0; i < nm; ++i) if (am[i] < 0 || cm[i] < 0) throw Error(DSRG_E_ARG, "negative stride");
    for (int i = 0; i < nn; ++i) if (bn[i] < 0 || cn[i] < 0) throw Error(DSRG_E_ARG, "negative stride");
    for (int i = 0; i < nk; ++i) if (ak[i] < 0 || bk[i] < 0) throw Error(DSRG_E_ARG, "negative stride");
    if (amax >= na || bmax >= nb || cmax >= nc) throw Error(DSRG_E_ARG, "strides address past the arrays");
    if (M >= (1LL << 31) || N >= (1LL << 31) || K >= (1LL << 31)) throw Error(DSRG_E_ARG, "too large");
    g.M = (int)M; g.N = (int)N; g.K = (int)K;
    gett_prepare(g);
    g.alpha = alpha; g.beta = beta ? 1 : 0;
    double *dA, *dB, *dC;
    HIPCHECK(hipMalloc(&dA, na * 8));
    HIPCHECK(hipMalloc(&dB, nb * 8));
    HIPCHECK(hipMalloc(&dC, nc * 8));
    HIPCHECK(hipMemcpy(dA, A, na * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dB, B, nb * 8, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(dC, C, nc * 8, hipMemcpyHostToDevice));
    // with a workspace, shapes with few output tiles and a long k range use split-K (room
    // for up to 8 partial outputs, at least 2^22 and at most 2^28 doubles)
    const long long ws_elems = std::max<long long>(1LL << 22, std::min<long long>(8LL * M * N, 1LL << 28));
    double* ws;
    HIPCHECK(hipMalloc(&ws, ws_elems * 8));
    launch_gett(g, dA, dB, dC, 0, kRoleGeneric, ws, ws_elems, precision);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipDeviceSynchronize());
    (void)hipFree(ws);
    HIPCHECK(hipMemcpy(C, dC, nc * 8, hipMemcpyDeviceToHost));
    (void)hipFree(dA); (void)hipFree(dB); (void)hipFree(dC);
    return DSRG_OK;
  });
}
