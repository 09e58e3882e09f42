// Device kernels of the DSRG-MRPT3 hot path for CDNA4 (gfx950), FP64.
#include "kernels.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

namespace dsrg {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Strided multi-index helpers
// ---------------------------------------------------------------------------
// Offset of the row-major multi-index idx over components d[0..n) with strides s.  The
// outermost component takes what is left of idx (idx < prod d), so it needs no division.
// Multi-index decode with each division a multiply-high and shift: for 1 <= d < 2^31 and
// l = ceil(log2 d), m = floor(2^(31+l) / d) + 1 < 2^32 gives floor(n / d) = (n m) >> (31 + l)
// for every 0 <= n < 2^31 (the error term n (m d - 2^(31+l)) / (d 2^(31+l)) < 2^-l <= 1/d
// cannot carry past the next multiple of d; Granlund and Montgomery, PLDI 1994).
__device__ __forceinline__ long long decode_fast(int idx, int n, const int* d, const unsigned* mag,
                                                 const int* sh, const long long* s) {
  long long off = 0;
#pragma unroll
  for (int c = kMaxComp - 1; c >= 1; --c) {
    if (c < n) {
      const int q = (int)(((unsigned long long)(unsigned)idx * mag[c]) >> sh[c]);
      const int r = idx - q * d[c];
      off += (long long)r * s[c];
      idx = q;
    }
  }
  if (n > 0) off += (long long)idx * s[0];
  return off;
}

__device__ __forceinline__ void decode2(long long idx, int n, const int* d, const long long* sa,
                                        const long long* sb, long long& oa, long long& ob) {
  oa = 0;
  ob = 0;
  for (int c = n - 1; c >= 0; --c) {
    long long q = idx / d[c];
    long long r = idx - q * d[c];
    oa += r * sa[c];
    ob += r * sb[c];
    idx = q;
  }
}

// the same for idx < 2^31 with the divisions as multiply and shift
// (the component loop is unrolled over the arrays' bound NC so the descriptor fields stay in
// registers across a caller's loop instead of being reloaded)
template <int NC>
__device__ __forceinline__ void decode2_fast(unsigned idx, int n, const int* d, const DivMagic& m,
                                             const long long* sa, const long long* sb, long long& oa,
                                             long long& ob) {
  oa = 0;
  ob = 0;
#pragma unroll
  for (int c = NC - 1; c >= 0; --c) {
    if (c < n) {
      const unsigned q = (unsigned)(((unsigned long long)idx * m.mag[c]) >> m.sh[c]);
      const long long r = (long long)(idx - q * (unsigned)d[c]);
      oa += r * sa[c];
      if (sb) ob += r * sb[c];
      idx = q;
    }
  }
}



// ---------------------------------------------------------------------------
// GETT: a workgroup of 256 threads (4 waves, 2x2) computes a BM x BN output tile; each
// wave owns a (16 WM) x (16 WN) sub-tile made of WM x WN v_mfma_f64_16x16x4 tiles.
// k advances in steps of BK = 16 values of the inner k component (zero-padded past its
// extent); the outer k components advance between steps, their base offsets carried in
// uniform registers, so a step's loads are plain base + per-thread-constant addresses.
// Steps are staged through LDS with two buffers: the next step's global loads are issued
// into registers before the current step's MFMAs and stored to the other buffer
// afterwards (one barrier per step).
// Operand layout of the 16x16x4 FP64 MFMA (checked on gfx950 by the kernel unit tests):
// lane l holds A[l%16][l/16] and B[l/16][l%16]; accumulator element r of lane l is
// D[l/16 + 4 r][l%16].
// ---------------------------------------------------------------------------
constexpr int BK = kGettBK;

// Tile of WGM x (4 / WGM) waves, each wave WM x WN MFMA blocks of 16 x 16; T is the
// element type staged in LDS (double, or float for the FP32-product precision).
template <int WM, int WN, int WGM, class T = double, int kBK = BK>
struct alignas(16) TileLds {
  static constexpr int BM = 16 * WM * WGM, BN = 16 * WN * (4 / WGM);
  // row pitch: 16 lanes of a 64-bit access (one bank pass) with k = 0..15 and one m land on
  // distinct banks when 2 pitch = 2 (mod 32 banks), i.e. an odd pitch of doubles; 32 lanes
  // of a 32-bit access with k = 0..15 and two m need a pitch of 2 (mod 32) floats (with 32
  // k values per step the slots still put k = 0..15 of two rows on 32 lanes).  The 128 x 128
  // FP64 tiles store rows m, m + 1 (m even) as one 16-byte access: 8 lanes per bank pass
  // with k = 0..7 are distinct with a pitch of 2 (mod 4) doubles, which keeps them aligned.
  static constexpr int PAD = sizeof(T) == 8 ? (BM == 128 && BN == 128 ? 2 : 1) : 2;
  static constexpr int LDA = BM + PAD, LDB = BN + PAD;
  T As[2][kBK * LDA];
  T Bs[2][kBK * LDB];
};

// MFMA blocks of the three precisions (kP = DSRG_PRECISION_*).  FP64 (0):
// v_mfma_f64_16x16x4f64, accumulator element r of lane l is D[l/16 + 4 r][l%16].  FP32
// products (1): v_mfma_f32_16x16x4f32 (operands rounded to FP32, products accumulated in
// FP32 for at most kF32FlushSteps k steps, then added into the FP64 output); accumulator
// element r of lane l is D[4 (l/16) + r][l%16].  Split BF16 x3 (2): each FP32-rounded
// operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a 16 x 16 x 16 block is
// hi.hi + hi.lo + lo.hi on v_mfma_f32_16x16x16bf16_1k with FP32 accumulation (lane l holds
// A[l%16][4 (l/16) + j] and B[4 (l/16) + j][l%16], j < 4; the accumulator as for FP32),
// flushed like FP32 products.
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
template <int kP>
struct Mfma;
template <>
struct Mfma<0> {
  using T = double;
  using Acc = double4_t;
  static __device__ __forceinline__ Acc zero() { return (Acc){0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ Acc fma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct Mfma<1> {
  using T = float;
  using Acc = float4_t;
  static __device__ __forceinline__ Acc zero() { return (Acc){0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ Acc fma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};
template <>
struct Mfma<2> {
  using T = float;
  using Acc = float4_t;
  static __device__ __forceinline__ Acc zero() { return (Acc){0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  // round to nearest even to BF16 (finite inputs); the BF16 bits
  static __device__ __forceinline__ unsigned short bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
  // x = hi + lo (+ a remainder below 2^-16 |x|)
  static __device__ __forceinline__ void split(float x, short& hi, short& lo) {
    const unsigned short h = bf16_bits(x);
    hi = (short)h;
    lo = (short)bf16_bits(x - __uint_as_float((unsigned)h << 16));
  }
  static __device__ __forceinline__ Acc fma3(short4_t ah, short4_t al, short4_t bh, short4_t bl, Acc c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
  }
};
constexpr int kF32FlushSteps = 64;

// One BM x BN output tile at (tile_m, tile_n) for chunk kz of the k steps of g.  kPackK:
// the tile supports packed k steps (g.kpack > 1); the 128 x 128 tiles leave it out (their
// launches are prepared without it) to keep their registers.
template <int WM, int WN, int WGM = 2, int kP = 0, bool kPackK = (WM * WN < 16), int kBK = BK>
__device__ __forceinline__ void gett_tile(const GettDesc& g, const double* __restrict__ A,
                                          const double* __restrict__ B, double* __restrict__ C,
                                          int tile_m, int tile_n, int kz,
                                          TileLds<WM, WN, WGM, typename Mfma<kP>::T, kBK>& lds) {
  using MF = Mfma<kP>;
  using T = typename MF::T;
  using Lds = TileLds<WM, WN, WGM, T, kBK>;
  constexpr int BK = kBK;   // k values per step of this tile
  constexpr int BM = Lds::BM, BN = Lds::BN;
  static_assert(BM * BK % 256 == 0 && BN * BK % 256 == 0 && 256 % BM == 0 || BM >= 256, "tile");
  static_assert(!kPackK || BK == kGettBK, "packed steps are prepared for the default step");
  constexpr int LDA = Lds::LDA, LDB = Lds::LDB;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;   // loads per thread per step
  // FP32 sums run over at most kF32FlushSteps default steps (1024 k values)
  constexpr int kFlushSteps = kF32FlushSteps * kGettBK / BK;
  auto& As = lds.As;
  auto& Bs = lds.Bs;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nk = g.nk;
  const int kin = g.kd[nk - 1];
  const long long a_in = g.ak[nk - 1], b_in = g.bk[nk - 1];
  const int ksteps = g.ksteps;
  // a step walks U values of component kw (the inner one, or with kpack the one before it,
  // whole inner ranges packed into the step); components below no advance between sweeps
  const int kp = kPackK ? g.kpack : 1;
  const int kw = kp > 1 ? nk - 2 : nk - 1;
  const int U = kp > 1 ? kp : BK;
  const int kdw = g.kd[kw];
  const long long a_st = g.ak[kw], b_st = g.bk[kw];
  const int no = kw;
  const long long s_lo = (long long)kz * g.kchunk;
  const long long s_hi = min(g.steps, s_lo + g.kchunk);
  const bool akf = g.a_kfast, bkf = g.b_kfast;

  // load slots: slot i of this thread covers (row, k) of the A tile and (k, col) of B.  With
  // k fastest, 16 lanes cover k = 0..15 of a row, slot i in row ma0 + 16 (i / kPair) at
  // k = ka0 + 16 (i % kPair) (kPair = BK / 16 slots per row); else every slot has the row
  // ma0 and k = ka0 + i kad.  The 128 x 128 tiles of plain launches (16 k per step in
  // FP64, 32 with FP32 / BF16 x3 products; kMPair) pair the rows instead: slots 2j and
  // 2j + 1 hold rows m and m + 1 at one k, written to LDS as one 16-byte (FP64) or 8-byte
  // store (k fastest: rows 2 (tid / 16) + q + 32 (i / (2 kPair)) at
  // k = tid % 16 + 16 ((i / 2) % kPair); else rows 2 (tid % 64) + q at
  // k = tid / 64 + 4 (i / 2)).  The per-slot values are one register plus uniform steps, so
  // the bounds tests and LDS addresses need no register per slot, and the operand offsets
  // one per row.
  constexpr int kPair = BK / kGettBK;
  static_assert(kPair * kGettBK == BK && 256 / kGettBK * kGettBK == 256, "slot rows");
  constexpr bool kMPair = BM == 128 && BN == 128 && !kPackK && BK == (kP != 0 ? 2 : 1) * kGettBK;
  const int ka0 = kMPair ? (akf ? (tid & 15) : tid >> 6) : (akf ? (tid & (kGettBK - 1)) : tid / BM);
  const int ma0 = kMPair ? (akf ? 2 * (tid >> 4) : 2 * (tid & 63)) : (akf ? tid / kGettBK : (tid & (BM - 1)));
  const int kb0 = kMPair ? (bkf ? (tid & 15) : tid >> 6) : (bkf ? (tid & (kGettBK - 1)) : tid / BN);
  const int nb0 = kMPair ? (bkf ? 2 * (tid >> 4) : 2 * (tid & 63)) : (bkf ? tid / kGettBK : (tid & (BN - 1)));
  const int kad = akf ? 0 : 256 / BM, kbd = bkf ? 0 : 256 / BN;
  // k and row (column) of slot i relative to (ka0, ma0)
  auto dk = [&](bool kf, int kd_, int i) -> int {
    if constexpr (kMPair) return kf ? 16 * ((i >> 1) % kPair) : 4 * (i >> 1);
    else return kf ? kGettBK * (i % kPair) : kd_ * i;
  };
  auto dm = [&](bool kf, int i) -> int {
    if constexpr (kMPair) return (i & 1) + (kf ? 32 * (i / (2 * kPair)) : 0);
    else return kf ? 256 / kGettBK * (i / kPair) : 0;
  };
  // operand rows held per thread and the first slot of row r (paired tiles, k fastest:
  // row r = 2 j + q holds slots 2 kPair j + q + 2 h)
  constexpr int kRows = kMPair ? 8 : (BM >= BN ? NA : NB) / kPair;
  auto first_of = [&](bool kf, int r) -> int {
    if constexpr (kMPair) return kf ? ((r & 1) | ((r >> 1) * 2 * kPair)) : (r & 1);
    else return r * kPair;
  };
  auto a_dk = [&](int i) { return dk(akf, kad, i); };
  auto b_dk = [&](int i) { return dk(bkf, kbd, i); };
  auto a_k = [&](int i) { return ka0 + a_dk(i); };
  auto a_m = [&](int i) { return ma0 + dm(akf, i); };
  auto b_k = [&](int i) { return kb0 + b_dk(i); };
  auto b_n = [&](int i) { return nb0 + dm(bkf, i); };
  // k slot j of a step: value j of the inner component (plain steps), or value j % kin of
  // the inner and j / kin of the walked component (packed steps).  Each slot keeps a 4-bit
  // code v (j; or j / kin, 15 past the packed ranges) and is real in a step while v < L
  // with L = kin - c BK (plain) or min(8, kd[kw] - c kpack) (packed), so no per-slot
  // limits stay in registers.
  static_assert(!kPackK || (NA <= 8 && NB <= 8), "slot codes");
  auto slot_off = [&](int j, long long s_in, long long s_w) -> long long {
    return kp > 1 ? (long long)(j % kin) * s_in + (long long)(j / kin) * s_w : (long long)j * s_in;
  };
  auto slot_code = [&](int j) -> unsigned { return kp > 1 ? (j < kp * kin ? (unsigned)(j / kin) : 15u) : (unsigned)j; };
  // operand offset of the first slot of each row (0 past M, N: such rows read a real
  // element and reach only outputs that are never written); slot i adds the uniform
  // (k of i - k of its row's first slot) times the inner stride
  static_assert(NA / kPair <= kRows && NB / kPair <= kRows, "rows");
  long long aoff[kRows], boff[kRows];
  unsigned acode = 0, bcode = 0;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = first_of(akf, r);
    const int m = tile_m + a_m(i);
    aoff[r] = i < NA && m < g.M ? decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.am) + slot_off(a_k(i), a_in, a_st) : 0;
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = first_of(bkf, r);
    const int n = tile_n + b_n(i);
    boff[r] = i < NB && n < g.N ? decode_fast(n, g.nn, g.nd, g.nmag, g.nsh, g.bn) + slot_off(b_k(i), b_in, b_st) : 0;
  }
  if constexpr (kPackK) {
#pragma unroll
    for (int i = 0; i < NA; ++i) acode |= slot_code(a_k(i)) << (4 * i);
#pragma unroll
    for (int i = 0; i < NB; ++i) bcode |= slot_code(b_k(i)) << (4 * i);
  }
  // (constant indices: the two layouts of the paired tiles are chosen by a select)
  auto a_off = [&](int i) -> long long {
    if constexpr (kMPair)
      return akf ? aoff[(i & 1) | ((i / (2 * kPair)) << 1)] + (long long)(16 * ((i >> 1) % kPair)) * a_in
                 : aoff[i & 1] + (long long)(4 * (i >> 1)) * a_in;
    else
      return aoff[i / kPair] + (long long)(a_dk(i) - a_dk(i / kPair * kPair)) * a_in;
  };
  auto b_off = [&](int i) -> long long {
    if constexpr (kMPair)
      return bkf ? boff[(i & 1) | ((i / (2 * kPair)) << 1)] + (long long)(16 * ((i >> 1) % kPair)) * b_in
                 : boff[i & 1] + (long long)(4 * (i >> 1)) * b_in;
    else
      return boff[i / kPair] + (long long)(b_dk(i) - b_dk(i / kPair * kPair)) * b_in;
  };
  // slot i of A (B) is real in the current step (L = real_slots()); without packed steps
  // the code is the slot itself
  auto real_a = [&](int i, int L) -> bool {
    if constexpr (kPackK) return (int)((acode >> (4 * i)) & 15u) < L;
    else return ka0 < L - a_dk(i);
  };
  auto real_b = [&](int i, int L) -> bool {
    if constexpr (kPackK) return (int)((bcode >> (4 * i)) & 15u) < L;
    else return kb0 < L - b_dk(i);
  };

  // uniform k state: inner step c, outer counters and the outer base offsets
  int c;
  int cnt[kMaxComp];
  long long abo = 0, bbo = 0;
  {
    long long o = s_lo / ksteps;
    c = (int)(s_lo - o * ksteps);
#pragma unroll
    for (int j = kMaxComp - 2; j >= 0; --j) {
      cnt[j] = 0;
      if (j < no) {
        const long long q = o / g.kd[j];
        cnt[j] = (int)(o - q * g.kd[j]);
        o = q;
        abo += cnt[j] * g.ak[j];
        bbo += cnt[j] * g.bk[j];
      }
    }
  }
  auto advance = [&]() {
    if (++c < ksteps) return;
    c = 0;
    bool carry = true;
#pragma unroll
    for (int j = kMaxComp - 2; j >= 0; --j) {
      if (carry && j < no) {
        ++cnt[j];
        abo += g.ak[j];
        bbo += g.bk[j];
        if (cnt[j] < g.kd[j]) {
          carry = false;
        } else {
          cnt[j] = 0;
          abo -= g.kd[j] * g.ak[j];
          bbo -= g.kd[j] * g.bk[j];
        }
      }
    }
  };

  auto real_slots = [&]() -> int { return kp > 1 ? min(8, kdw - c * kp) : kin - c * BK; };
  double ra[NA], rb[NB];
  // loads of the step (c): out-of-range slots read the step's first element (valid) and
  // are zeroed by the select in stash, which runs after the MFMAs so the loads overlap them
  auto fetch = [&]() {
    const int k0 = c * U;
    const int L = real_slots();
    const long long ab = abo + k0 * a_st, bb = bbo + k0 * b_st;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const bool ok = real_a(i, L);
      ra[i] = A[ab + (ok ? a_off(i) : 0)];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const bool ok = real_b(i, L);
      rb[i] = B[bb + (ok ? b_off(i) : 0)];
    }
  };
  // rows (columns) past M (N) hold a real element of the operand (offset 0): they only
  // reach output rows (columns) that are never written, so only the k range is masked
  const int a_l0 = ka0 * LDA + ma0, b_l0 = kb0 * LDB + nb0;
  auto stash = [&](int buf) {
    const int L = real_slots();
    if constexpr (kMPair) {
      // rows m, m + 1 (m even; even pitch) at one k: one store per pair
      typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int i = 0; i < NA; i += 2) {
        const bool ok = real_a(i, L);
        *(T2*)&As[buf][a_l0 + a_dk(i) * LDA + dm(akf, i)] = (T2){ok ? (T)ra[i] : (T)0, ok ? (T)ra[i + 1] : (T)0};
      }
#pragma unroll
      for (int i = 0; i < NB; i += 2) {
        const bool ok = real_b(i, L);
        *(T2*)&Bs[buf][b_l0 + b_dk(i) * LDB + dm(bkf, i)] = (T2){ok ? (T)rb[i] : (T)0, ok ? (T)rb[i + 1] : (T)0};
      }
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i)
        As[buf][a_l0 + a_dk(i) * LDA + dm(akf, i)] = real_a(i, L) ? (T)ra[i] : (T)0;
#pragma unroll
      for (int i = 0; i < NB; ++i)
        Bs[buf][b_l0 + b_dk(i) * LDB + dm(bkf, i)] = real_b(i, L) ? (T)rb[i] : (T)0;
    }
  };

  typename MF::Acc acc[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) acc[a][b] = MF::zero();

  const int wm = (wave % WGM) * (16 * WM);
  const int wn = (wave / WGM) * (16 * WN);
  const int li = lane & 15;
  const int lk = lane >> 4;

  // write the accumulators: the first write of a tile follows beta (split-K partial tiles
  // are written plain), later writes (FP32 products only) add to what is there
  auto flush = [&](bool first) {
    // an opaque copy of the tile origin keeps the compiler from hoisting the output
    // offsets of every row and column out of the k loop (they would stay live in VGPRs)
    int tm0 = tile_m, tn0 = tile_n;
    asm volatile("" : "+v"(tm0), "+v"(tn0));
#pragma unroll
    for (int a = 0; a < WM; ++a) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = tm0 + wm + a * 16 + MF::row(lk, r);
        if (m >= g.M) continue;
        if (g.part) {
          const long long pM = g.pM ? g.pM : g.M, pN = g.pM ? g.pN : g.N;
          double* prow = g.part + ((long long)kz * pM + (m - g.pm0)) * pN - g.pn0;
#pragma unroll
          for (int b = 0; b < WN; ++b) {
            int n = tn0 + wn + b * 16 + li;
            if (n < g.N) prow[n] = first ? (double)acc[a][b][r] : prow[n] + (double)acc[a][b][r];
          }
          continue;
        }
        long long cmo = decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.cm);
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          int n = tn0 + wn + b * 16 + li;
          if (n >= g.N) continue;
          long long o = cmo + decode_fast(n, g.nn, g.nd, g.nmag, g.nsh, g.cn);
          double v = g.alpha * (double)acc[a][b][r];
          if (g.beta || !first) v += C[o];
          C[o] = v;
        }
      }
    }
  };

  int buf = 0;
  if (s_lo < s_hi) {
    fetch();
    stash(0);
  }
  __syncthreads();
  bool first = true;
  int since = 0;
  // the MFMAs of one step on LDS buffer buf
  auto compute = [&]() {
    if constexpr (kP == 2) {
      // 16-deep BF16 blocks: in block h lane (li, lk) splits k = 16 h + 4 lk .. + 3 of its
      // row (column) into hi and lo parts
      static_assert(BK % 16 == 0, "whole BF16 blocks per step");
#pragma unroll
      for (int h16 = 0; h16 < BK; h16 += 16) {
        short4_t ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
        for (int t = 0; t < WM; ++t)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            short h, l;
            MF::split(As[buf][(h16 + 4 * lk + j) * LDA + wm + t * 16 + li], h, l);
            ah[t][j] = h;
            al[t][j] = l;
          }
#pragma unroll
        for (int t = 0; t < WN; ++t)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            short h, l;
            MF::split(Bs[buf][(h16 + 4 * lk + j) * LDB + wn + t * 16 + li], h, l);
            bh[t][j] = h;
            bl[t][j] = l;
          }
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
          for (int b = 0; b < WN; ++b) acc[a][b] = MF::fma3(ah[a], al[a], bh[b], bl[b], acc[a][b]);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        T av[WM], bv[WN];
#pragma unroll
        for (int t = 0; t < WM; ++t) av[t] = As[buf][(kk + lk) * LDA + wm + t * 16 + li];
#pragma unroll
        for (int t = 0; t < WN; ++t) bv[t] = Bs[buf][(kk + lk) * LDB + wn + t * 16 + li];
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
          for (int b = 0; b < WN; ++b) acc[a][b] = MF::fma(av[a], bv[b], acc[a][b]);
      }
    }
  };
  // every step but the last loads the next one (the last is peeled off, so the loop's
  // loads are always waited for inside the loop)
  long long s = s_lo;
  for (; s + 1 < s_hi; ++s) {
    advance();
    fetch();
    compute();
    if (kP != 0 && ++since == kFlushSteps) {
      flush(first);
      first = false;
      since = 0;
#pragma unroll
      for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) acc[a][b] = MF::zero();
    }
    stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (s < s_hi) {
    compute();
    __syncthreads();
  }
  flush(first);
}

// Workgroups are dispatched to the 8 XCDs round-robin by their id; this bijection gives
// XCD x a contiguous range of logical tiles, so the tiles that share operand panels share
// one XCD's L2 instead of being spread over all eight.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int q = total / kXcds, r = total - q * kXcds;
  const int x = b % kXcds, j = b / kXcds;
  return x * q + min(x, r) + j;
}

// Grouped launches order their tiles longest first; a contiguous range per XCD would load
// XCD 0 with the longest ones.  Within each window of kXcds * 8 workgroups XCD x takes 8
// consecutive tiles instead (the tail past the last whole window keeps its order).
__device__ __forceinline__ int xcd_tile_windowed(int b, int total) {
  constexpr int c = 8, W = kXcds * c;
  const int full = total / W * W;
  if (b >= full) return b;
  const int base = b / W * W, o = b - base;
  return base + (o % kXcds) * c + o / kXcds;
}

// Tile (tm, tn) of logical index Lp among the gx x gy tiles of one k split: groups of
// kGroupM m tiles, each group walked m fastest and then n.  Consecutive indices go to one
// XCD (xcd_tile), so the workgroups resident on an XCD at one time cover a block of about
// kGroupM m tiles by (resident / kGroupM) n tiles and share both operands' panels in its L2,
// instead of one column of m tiles that shares only the B panel.
constexpr int kGroupM = 8;
__device__ __forceinline__ void grouped_tile(int Lp, int gx, int gy, int& tm, int& tn) {
  const int per = kGroupM * gy;
  const int gid = Lp / per;
  const int first = gid * kGroupM;
  const int gsz = min(gx - first, kGroupM);
  const int r = Lp - gid * per;
  tm = first + r % gsz;
  tn = r / gsz;
}

// Logical tile L of a (gx, gy, gz) grid (grouped m tiles, see grouped_tile; plain m-first
// order with the triangle skip).
template <int WM, int WN, int kP, int kBK, int WGM = 2>
__device__ __forceinline__ void gett_grid_tile(const GettDesc& g, const double* __restrict__ A,
                                               const double* __restrict__ B, double* __restrict__ C,
                                               TileLds<WM, WN, WGM, typename Mfma<kP>::T, kBK>& lds) {
  using Lds = TileLds<WM, WN, WGM, typename Mfma<kP>::T, kBK>;
  constexpr int BM = Lds::BM, BN = Lds::BN;
  // a tail launch covers logical tiles [t0, t0 + nl) of the gx x gy grid in g
  const bool sub = g.gx > 0;
  const int gx = sub ? g.gx : gridDim.x, gy = sub ? g.gy : gridDim.y;
  const int nl = sub ? g.nl : gx * gy;
  const int total = gridDim.x * gridDim.y * gridDim.z;
  const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  // with the triangle skip the live tiles crowd into the last columns: runs of 8 tiles
  // spread over the XCDs keep their loads even
  const int L = g.tri > 0 ? xcd_tile_windowed(b, total) : xcd_tile(b, total);
  int tm, tn, kz;
  if (g.tri > 0) {
    tm = L % gx;
    const int rest = L / gx;
    tn = rest % gy;
    kz = rest / gy;
  } else {
    kz = L / nl;
    grouped_tile(g.t0 + L - kz * nl, gx, gy, tm, tn);
  }
  if (g.tri > 0 && (tn * BN + BN - 1) / g.tri < (tm * BM) / g.tri) return;
  gett_tile<WM, WN, WGM, kP, (WM * WN < 16), kBK>(g, A, B, C, tm * BM, tn * BN, kz, lds);
}

// k values per step of the plain launches: FP32 and BF16 x3 products on 128 x 128 tiles
// walk 32 (the FP32 LDS tiles of two steps fit where one FP64 step does, and each barrier
// and LDS write pass then feeds twice the MFMAs), everything else kGettBK
template <int kP, int WM, int WN>
constexpr int plain_bk() { return kP != 0 && WM * WN == 16 ? kGettBigBK : kGettBK; }

// WGM: waves along m (2: 64 x 64 and 128 x 128 tiles; 4: 128 x 32 tiles of skinny outputs)
template <int kRole, int WM, int WN, int WGM = 2>
__global__ __launch_bounds__(256) void gett_f64_kernel(GettDesc g, const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       double* __restrict__ C) {
  __shared__ TileLds<WM, WN, WGM, double, plain_bk<0, WM, WN>()> lds;
  gett_grid_tile<WM, WN, 0, plain_bk<0, WM, WN>(), WGM>(g, A, B, C, lds);
}

// FP64 operands and output, FP32 products (DSRG_PRECISION_FP32); two workgroups per CU
// (the 32-deep steps of the 128 x 128 tiles would otherwise take every register)
template <int kRole, int WM, int WN, int WGM = 2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gett_f32_kernel(GettDesc g, const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       double* __restrict__ C) {
  __shared__ TileLds<WM, WN, WGM, float, plain_bk<1, WM, WN>()> lds;
  gett_grid_tile<WM, WN, 1, plain_bk<1, WM, WN>(), WGM>(g, A, B, C, lds);
}

// FP64 operands and output, split-BF16 x3 products (DSRG_PRECISION_BF16X3); two
// workgroups per CU as for FP32 products
template <int kRole, int WM, int WN, int WGM = 2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gett_b3_kernel(GettDesc g, const double* __restrict__ A,
                                                      const double* __restrict__ B,
                                                      double* __restrict__ C) {
  __shared__ TileLds<WM, WN, WGM, float, plain_bk<2, WM, WN>()> lds;
  gett_grid_tile<WM, WN, 2, plain_bk<2, WM, WN>(), WGM>(g, A, B, C, lds);
}

// C[m][n] = alpha * sum_z part[z][m][n] (+ C) in a fixed order of z
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GettDesc g, const double* __restrict__ part,
                                                            int nsplit, double* __restrict__ C) {
  long long total = (long long)g.M * g.N;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < total; i += 256LL * gridDim.x) {
    int m = (int)(i / g.N), n = (int)(i - (long long)m * g.N);
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[(long long)z * total + i];
    long long o = decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.cm) + decode_fast(n, g.nn, g.nd, g.nmag, g.nsh, g.cn);
    double v = g.alpha * s;
    if (g.beta) v += C[o];
    C[o] = v;
  }
}

// The k-split tail of a 128 x 128 launch: C[m][n] = alpha * sum_z part[z][m - pm0][n - pn0]
// (+ C) in a fixed order of z, for the elements of the box whose tile is one of the tail's
// (logical index >= t0: the inverse of grouped_tile); the others were written by the main
// launch.
__global__ __launch_bounds__(256) void splitk_tail_reduce_kernel(GettDesc g, const double* __restrict__ part,
                                                                 int nsplit, double* __restrict__ C) {
  const long long box = (long long)g.pM * g.pN;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < box; i += 256LL * gridDim.x) {
    const int m = g.pm0 + (int)(i / g.pN), n = g.pn0 + (int)(i % g.pN);
    const int tm = m / 128, tn = n / 128;
    const int first = tm / kGroupM * kGroupM, gsz = min(g.gx - first, kGroupM);
    if (first * g.gy + tn * gsz + (tm - first) < g.t0) continue;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[(long long)z * box + i];
    const long long o = decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.cm) + decode_fast(n, g.nn, g.nd, g.nmag, g.nsh, g.cn);
    double v = g.alpha * s;
    if (g.beta) v += C[o];
    C[o] = v;
  }
}

// Merge k components that are contiguous in both operands (the outer one's strides are
// the inner one's times its extent), then move to the last place the inner component:
// first the one that lets most operands load coalesced (unit k stride, or a unit stride of
// the operand's innermost free index), then the one whose padding to whole steps wastes
// least, then the larger.
// Merge free components that are contiguous in both the operand and C: outer i, inner j
// with s_op[i] == d[j] s_op[j] and s_c[i] == d[j] s_c[j] become one component (fewer
// divisions in every index decode).
static void merge_free(int& n, int* d, long long* so, long long* sc) {
  for (bool merged = true; merged && n > 1;) {
    merged = false;
    for (int i = 0; i + 1 < n && !merged; ++i) {
      const int j = i + 1;
      if (so[i] == (long long)d[j] * so[j] && sc[i] == (long long)d[j] * sc[j]) {
        d[j] *= d[i];
        for (int t = i; t + 1 < n; ++t) {
          d[t] = d[t + 1];
          so[t] = so[t + 1];
          sc[t] = sc[t + 1];
        }
        --n;
        merged = true;
      }
    }
  }
}

static void magic_of(int d, unsigned& m, int& sh) {
  int l = 0;
  while (l < 31 && (1LL << l) < (long long)d) ++l;
  sh = 31 + l;
  m = (unsigned)((1ULL << sh) / (unsigned long long)std::max(d, 1) + 1);
}

void gett_magic(GettDesc& g) {
  for (int c = 0; c < kMaxComp; ++c) {
    magic_of(c < g.nm ? g.md[c] : 1, g.mmag[c], g.msh[c]);
    magic_of(c < g.nn ? g.nd[c] : 1, g.nmag[c], g.nsh[c]);
  }
}

static bool big_tiles(const GettDesc& g);

double gett_tile_fraction(const GettDesc& g) {
  if (g.tri <= 0 || g.M <= 0 || g.N <= 0) return 1.0;
  const int b = big_tiles(g) ? 128 : 64;
  double done = 0;
  for (int tm = 0; tm < g.M; tm += b)
    for (int tn = 0; tn < g.N; tn += b)
      if ((tn + b - 1) / g.tri >= tm / g.tri)
        done += (double)std::min(b, g.M - tm) * std::min(b, g.N - tn);
  return done / ((double)g.M * g.N);
}

void gett_unpack_k(GettDesc& g) {
  if (g.kpack <= 1) return;
  const int kin = g.kd[g.nk - 1];
  g.kpack = 1;
  g.ksteps = (kin + BK - 1) / BK;
  g.steps = (long long)(g.K / kin) * g.ksteps;
  g.kchunk = g.steps;
}

void gett_prepare(GettDesc& g) {
  merge_free(g.nm, g.md, g.am, g.cm);
  merge_free(g.nn, g.nd, g.bn, g.cn);
  if (g.nk == 0) {
    g.nk = 1;
    g.kd[0] = 1;
    g.ak[0] = 0;
    g.bk[0] = 0;
  }
  for (bool merged = true; merged && g.nk > 1;) {
    merged = false;
    for (int i = 0; i < g.nk && !merged; ++i)
      for (int j = 0; j < g.nk && !merged; ++j) {
        if (i == j) continue;
        if (g.ak[i] == (long long)g.kd[j] * g.ak[j] && g.bk[i] == (long long)g.kd[j] * g.bk[j]) {
          // i is the outer of the pair: (i, j) -> one component with j's strides
          g.kd[j] *= g.kd[i];
          for (int t = i; t + 1 < g.nk; ++t) {
            g.kd[t] = g.kd[t + 1];
            g.ak[t] = g.ak[t + 1];
            g.bk[t] = g.bk[t + 1];
          }
          --g.nk;
          merged = true;
        }
      }
  }
  auto waste = [&](int j) { return (double)((g.kd[j] + BK - 1) / BK * BK) / g.kd[j]; };
  const bool am1 = g.nm > 0 && std::llabs(g.am[g.nm - 1]) == 1;
  const bool bn1 = g.nn > 0 && std::llabs(g.bn[g.nn - 1]) == 1;
  auto coalesced = [&](int j) {
    return (int)(am1 || std::llabs(g.ak[j]) == 1) + (int)(bn1 || std::llabs(g.bk[j]) == 1);
  };
  int best = g.nk - 1;
  for (int j = 0; j < g.nk; ++j) {
    const int cj = coalesced(j), cb = coalesced(best);
    const double wj = waste(j), wb = waste(best);
    if (cj > cb || (cj == cb && (wj < wb - 1e-12 || (wj <= wb + 1e-12 && g.kd[j] > g.kd[best]))))
      best = j;
  }
  std::swap(g.kd[best], g.kd[g.nk - 1]);
  std::swap(g.ak[best], g.ak[g.nk - 1]);
  std::swap(g.bk[best], g.bk[g.nk - 1]);
  const int kin = g.kd[g.nk - 1];
  g.kpack = 1;
  g.ksteps = (kin + BK - 1) / BK;
  g.steps = (long long)(g.K / kin) * g.ksteps;
  if (g.nk >= 2 && 2 * kin <= BK) {
    // pack whole inner ranges into a step along the outer component that pads least
    // (ties: the larger); keep it only if it saves steps
    const int R = BK / kin;
    int o = 0;
    auto pad = [&](int j) { return (double)((g.kd[j] + R - 1) / R * R) / g.kd[j]; };
    for (int j = 1; j < g.nk - 1; ++j)
      if (pad(j) < pad(o) - 1e-12 || (pad(j) <= pad(o) + 1e-12 && g.kd[j] > g.kd[o])) o = j;
    const long long ksp = (g.kd[o] + R - 1) / R;
    const long long stp = (long long)(g.K / ((long long)kin * g.kd[o])) * ksp;
    if (stp < g.steps) {
      std::swap(g.kd[o], g.kd[g.nk - 2]);
      std::swap(g.ak[o], g.ak[g.nk - 2]);
      std::swap(g.bk[o], g.bk[g.nk - 2]);
      g.kpack = R;
      g.ksteps = (int)ksp;
      g.steps = stp;
    }
  }
  if (big_tiles(g)) gett_unpack_k(g);   // 128 x 128 launches walk plain steps
  g.kchunk = g.steps;
  g.part = nullptr;
  const long long ai = std::llabs(g.ak[g.nk - 1]), bi = std::llabs(g.bk[g.nk - 1]);
  g.a_kfast = g.nm == 0 || ai < std::llabs(g.am[g.nm - 1]);
  g.b_kfast = g.nn == 0 || bi < std::llabs(g.bn[g.nn - 1]);
  gett_magic(g);
}

// Large tiles (128 x 128) when they still give enough workgroups, else 64 x 64.
// per host thread: a call plans and launches its contractions on one thread
static thread_local int t_big_tile_min = 256;
void set_big_tile_min(int n) { t_big_tile_min = n > 0 ? n : 256; }
int big_tile_min() { return t_big_tile_min; }

static bool big_tiles(const GettDesc& g) {
  long long t128 = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128);
  return g.M >= 128 && g.N >= 128 && t128 >= t_big_tile_min && g.steps >= g.big_min_steps;
}

bool gett_big_tiles(const GettDesc& g) { return big_tiles(g); }

// 128 x 32 tiles (four waves along m) for plain launches with at most 32 output columns and
// many rows: a 64 x 64 tile there computes more than half of its MFMA work on zero columns.
// Also for long k ranges over at least 256 rows (reductions such as 308 x 28 x 2.7e6):
// fewer m tiles each stream the whole B operand.
static bool skinny_tiles(const GettDesc& g) {
  return !big_tiles(g) && g.tri <= 0 && g.N <= 32 && (g.M >= 2048 || (g.M >= 256 && g.steps >= 4096));
}

// k-split tail of a 128 x 128 launch with more tiles than the 512 resident workgroup slots
// (two per CU) whose last round is at most half full: the last rem logical tiles would run
// alone for a whole tile time, so their k range is split smax ways instead (rem x smax about
// one round; the launcher lowers the split to keep 16 k steps per chunk).  Only tails inside
// the last group of kGroupM m tiles (grouped_tile), whose partial tiles are kept over the
// box of rows from that group's first and columns from the tail's first, at most
// kTailCap doubles.
constexpr long long kTailCap = 1LL << 24;
struct TailPlan {
  int gx = 0, gy = 0, t0 = 0, rem = 0, smax = 0;
  int pm0 = 0, pn0 = 0, pM = 0, pN = 0;
};
static TailPlan tail_plan(const GettDesc& g) {
  TailPlan t;
  if (!big_tiles(g) || g.tri > 0) return t;
  const int gx = (g.M + 127) / 128, gy = (g.N + 127) / 128;
  const long long tiles = (long long)gx * gy, slots = 512;
  const int rem = (int)(tiles % slots);
  if (tiles <= slots || rem == 0 || rem > slots / 2 || tiles >= (1LL << 31)) return t;
  const int first = (gx - 1) / kGroupM * kGroupM, gsz = gx - first;
  if ((long long)rem > (long long)gsz * gy) return t;
  const int tn_lo = (gsz * gy - rem) / gsz;
  const int pm0 = first * 128, pn0 = tn_lo * 128, pM = g.M - pm0, pN = g.N - pn0;
  long long s = std::min<long long>(32, slots / rem);
  while (s >= 2 && s * pM * pN > kTailCap) --s;
  if (s < 2) return t;
  t.gx = gx; t.gy = gy; t.t0 = (int)(tiles - rem); t.rem = rem; t.smax = (int)s;
  t.pm0 = pm0; t.pn0 = pn0; t.pM = pM; t.pN = pN;
  return t;
}

long long gett_tail_ws(const GettDesc& g) {
  const TailPlan t = tail_plan(g);
  return t.rem ? (long long)t.smax * t.pM * t.pN : 0;
}

// Split-K factor: the number of k chunks that fills the resident workgroup slots in the
// most nearly whole rounds (256 CUs; two 128 x 128 or four 64 x 64 workgroups per CU fit
// the registers), keeping at least 16 k steps per chunk (4 when the output has at most
// 2^20 elements: there a few tiles with long k ranges would wait on load latency, and the
// partial tiles stay small) and the partial tiles within ws_elems.
//  - 64 x 64 tiles: a larger split must gain at least 5 % of utilisation.
//  - 128 x 128 tiles: the split with the least modelled time, rounds x (k steps per chunk
//    x 5.1 us + 8 us per tile) plus the partial tiles' HBM traffic (written and read
//    once, 16 bytes per element at 4 TB/s); the step and tile costs are the measured ones
//    of this kernel at two workgroups per CU.  Up to 64 chunks.  (Triangular launches,
//    whose grid skips tiles, keep the 5 % rule.)
int gett_splits(const GettDesc& g, long long ws_elems) {
  const bool big = big_tiles(g), skinny = skinny_tiles(g);
  const int bm = big || skinny ? 128 : 64, bn = big ? 128 : skinny ? 32 : 64;
  // resident workgroups per CU: registers (128 x 128), LDS (128 x 32: 41.5 KB), else 4
  const long long slots = 256LL * (big ? 2 : skinny ? 3 : 4);
  const long long tiles = (long long)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  const long long mn = std::max<long long>(1, (long long)g.M * g.N);
  const long long min_chunk = mn <= (1LL << 20) ? 4 : 16;
  const long long smax = std::min<long long>({g.steps / min_chunk, ws_elems / mn, 4096});
  if (big && g.tri <= 0) {
    auto model = [&](long long s) {
      const long long chunk = (g.steps + s - 1) / s;
      const long long w = tiles * ((g.steps + chunk - 1) / chunk);
      const double rounds = (double)((w + slots - 1) / slots);
      return rounds * ((double)chunk * 5.1e-6 + 8e-6) + (s > 1 ? (double)s * mn * 16.0 / 4e12 : 0.0);
    };
    long long best = 1;
    double tb = model(1);
    for (long long s = 2; s <= std::min<long long>(smax, 64); ++s) {
      const double t = model(s);
      if (t < tb) {
        best = s;
        tb = t;
      }
    }
    return (int)best;
  }
  auto util = [&](long long s) {
    const long long w = tiles * s;
    return (double)w / (double)(slots * ((w + slots - 1) / slots));
  };
  long long best = 1;
  double ub = util(1);
  for (long long s = 2; s <= smax && tiles * (s - 1) < 8 * slots; ++s) {
    const double u = util(s);
    if (u > ub + 0.05) {
      best = s;
      ub = u;
    }
  }
  return (int)best;
}

// shape: 0 64 x 64, 1 128 x 128, 2 128 x 32 tiles
template <int kRole>
static void launch_role(const GettDesc& g, int shape, int prec, dim3 grid, const double* A,
                        const double* B, double* C, hipStream_t st) {
  if (prec == 2) {
    if (shape == 1)
      hipLaunchKernelGGL((gett_b3_kernel<kRole, 4, 4>), grid, dim3(256), 0, st, g, A, B, C);
    else if (shape == 2)
      hipLaunchKernelGGL((gett_b3_kernel<kRole, 2, 2, 4>), grid, dim3(256), 0, st, g, A, B, C);
    else
      hipLaunchKernelGGL((gett_b3_kernel<kRole, 2, 2>), grid, dim3(256), 0, st, g, A, B, C);
  } else if (prec == 1) {
    if (shape == 1)
      hipLaunchKernelGGL((gett_f32_kernel<kRole, 4, 4>), grid, dim3(256), 0, st, g, A, B, C);
    else if (shape == 2)
      hipLaunchKernelGGL((gett_f32_kernel<kRole, 2, 2, 4>), grid, dim3(256), 0, st, g, A, B, C);
    else
      hipLaunchKernelGGL((gett_f32_kernel<kRole, 2, 2>), grid, dim3(256), 0, st, g, A, B, C);
  } else {
    if (shape == 1)
      hipLaunchKernelGGL((gett_f64_kernel<kRole, 4, 4>), grid, dim3(256), 0, st, g, A, B, C);
    else if (shape == 2)
      hipLaunchKernelGGL((gett_f64_kernel<kRole, 2, 2, 4>), grid, dim3(256), 0, st, g, A, B, C);
    else
      hipLaunchKernelGGL((gett_f64_kernel<kRole, 2, 2>), grid, dim3(256), 0, st, g, A, B, C);
  }
}

void launch_gett(const GettDesc& g0, const double* A, const double* B, double* C, hipStream_t st,
                 int role, double* ws, long long ws_elems, int prec) {
  if (g0.M <= 0 || g0.N <= 0) return;
  GettDesc g = g0;
  gett_magic(g);
  const bool big = big_tiles(g);
  if (big) gett_unpack_k(g);
  if (big && prec != 0) {
    // these kernels walk kGettBigBK k values per step
    const int kin = g.kd[g.nk - 1];
    g.ksteps = (kin + kGettBigBK - 1) / kGettBigBK;
    g.steps = (long long)(g.K / kin) * g.ksteps;
    g.kchunk = g.steps;
  }
  const int shape = big ? 1 : skinny_tiles(g) ? 2 : 0;
  const int bm = shape ? 128 : 64, bn = shape == 1 ? 128 : shape == 2 ? 32 : 64;
  int ns = ws ? gett_splits(g, ws_elems) : 1;
  g.part = nullptr;
  g.kchunk = g.steps;
  if (ns == 1 && ws && big) {
    const TailPlan t = tail_plan(g);
    long long s = std::min<long long>(t.smax, g.steps / 16);
    if (t.rem > 0 && s >= 2 && s * t.pM * t.pN <= ws_elems) {
      // the whole rounds in one launch, the tail's k chunks in another, then the tail's
      // fixed-order reduction
      GettDesc gm = g;
      gm.gx = t.gx; gm.gy = t.gy; gm.t0 = 0; gm.nl = t.t0;
      GettDesc gt = g;
      gt.gx = t.gx; gt.gy = t.gy; gt.t0 = t.t0; gt.nl = t.rem;
      const long long chunk = (g.steps + s - 1) / s;
      const int nz = (int)((g.steps + chunk - 1) / chunk);
      gt.kchunk = chunk;
      gt.part = ws;
      gt.pm0 = t.pm0; gt.pn0 = t.pn0; gt.pM = t.pM; gt.pN = t.pN;
      auto go = [&](const GettDesc& d, dim3 grid) {
        if (role == kRoleLadder)
          launch_role<kRoleLadder>(d, shape, prec, grid, A, B, C, st);
        else if (role == kRoleIntegrals)
          launch_role<kRoleIntegrals>(d, shape, prec, grid, A, B, C, st);
        else
          launch_role<kRoleGeneric>(d, shape, prec, grid, A, B, C, st);
      };
      go(gm, dim3((unsigned)t.t0, 1, 1));
      go(gt, dim3((unsigned)t.rem, 1, (unsigned)nz));
      const long long box = (long long)t.pM * t.pN;
      const long long blocks = std::min<long long>((box + 255) / 256, 4096);
      hipLaunchKernelGGL(splitk_tail_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, gt, ws, nz, C);
      return;
    }
  }
  if (ns > 1) {
    long long chunk = (g.steps + ns - 1) / ns;
    ns = (int)((g.steps + chunk - 1) / chunk);
    g.kchunk = chunk;
    g.part = ws;
  }
  dim3 grid((g.M + bm - 1) / bm, (g.N + bn - 1) / bn, ns);
  // the role only selects a distinct kernel symbol so profiles can tell the launches apart
  if (role == kRoleLadder)
    launch_role<kRoleLadder>(g, shape, prec, grid, A, B, C, st);
  else if (role == kRoleIntegrals)
    launch_role<kRoleIntegrals>(g, shape, prec, grid, A, B, C, st);
  else
    launch_role<kRoleGeneric>(g, shape, prec, grid, A, B, C, st);
  if (ns > 1) {
    long long total = (long long)g.M * g.N;
    long long blocks = std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, g, ws, ns, C);
  }
}

// ---------------------------------------------------------------------------
// Grouped contractions: independent GETTs of one dependency level in a single launch.
// Workgroup b finds its item by binary search over the items' first workgroups; items
// never share an output element, so the launch is race-free and its result does not
// depend on scheduling.
// ---------------------------------------------------------------------------
// Shape-4 items (K <= 16, N <= 64): the k offsets and B (zero past K and N) are staged in
// LDS, each thread loads the K values of its row of A and forms its N outputs in FP64
// (k in order), so a workgroup covers 256 rows at the cost of a streaming pass.
struct RowLds {
  double Bs[BK][kGroupRowN];
  long long ka[BK], kb[BK];
};
__device__ __forceinline__ void group_rows(const GroupItem& it, int tm, RowLds& lds) {
  const GettDesc& g = it.g;
  const int t = threadIdx.x;
  if (t < g.K) {
    long long oa = 0, ob = 0;
    int idx = t;
    for (int c = g.nk - 1; c >= 0; --c) {
      const int q = idx / g.kd[c];
      const int r = idx - q * g.kd[c];
      oa += (long long)r * g.ak[c];
      ob += (long long)r * g.bk[c];
      idx = q;
    }
    lds.ka[t] = oa;
    lds.kb[t] = ob;
  }
  __syncthreads();
  for (int e = t; e < BK * kGroupRowN; e += 256) {
    const int k = e / kGroupRowN, n = e % kGroupRowN;
    double v = 0.0;
    if (k < g.K && n < g.N) v = it.B[lds.kb[k] + decode_fast(n, g.nn, g.nd, g.nmag, g.nsh, g.bn)];
    lds.Bs[k][n] = v;
  }
  __syncthreads();
  const int m = tm * kGroupRows + t;
  if (m >= g.M) return;
  const long long ao = decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.am);
  double a[BK];
#pragma unroll
  for (int k = 0; k < BK; ++k) a[k] = k < g.K ? it.A[ao + lds.ka[k]] : 0.0;
  const long long co = decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.cm);
  for (int n = 0; n < g.N; ++n) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BK; ++k) s = fma(a[k], lds.Bs[k][n], s);
    double* c = it.C + co + decode_fast(n, g.nn, g.nd, g.nmag, g.nsh, g.cn);
    const double v = g.alpha * s;
    *c = g.beta ? *c + v : v;
  }
}

template <int kP>
__device__ __forceinline__ void group_tile(const GroupItem* __restrict__ items, const int* __restrict__ tile_item) {
  using T = typename Mfma<kP>::T;
  using GroupLds0 = TileLds<2, 2, 2, T>;
  using GroupLds1 = TileLds<1, 2, 1, T>;
  using GroupLds2 = TileLds<2, 1, 4, T>;
  static_assert(GroupLds0::BM == 64 && GroupLds0::BN == 64, "group tile 0");
  static_assert(GroupLds1::BM == 16 && GroupLds1::BN == 128, "group tile 1");
  static_assert(GroupLds2::BM == 128 && GroupLds2::BN == 16, "group tile 2");
  __shared__ union {
    GroupLds0 t0;
    GroupLds1 t1;
    GroupLds2 t2;
    RowLds rows;
  } lds;
  const int b = xcd_tile_windowed(blockIdx.x, gridDim.x);
  const GroupItem& it = items[tile_item[b]];
  const int t = b - it.tile0;
  const int per = it.tiles_m * it.tiles_n;
  const int kz = t / per;
  const int r = t - kz * per;
  const int tm = r / it.tiles_n;
  const int tn = r - tm * it.tiles_n;
  switch (it.shape) {
    case kGroupRowShape:
      group_rows(it, tm, lds.rows);
      break;
    case 1:
      gett_tile<1, 2, 1, kP>(it.g, it.A, it.B, it.C, tm * GroupLds1::BM, tn * GroupLds1::BN, kz, lds.t1);
      break;
    case 2:
      gett_tile<2, 1, 4, kP>(it.g, it.A, it.B, it.C, tm * GroupLds2::BM, tn * GroupLds2::BN, kz, lds.t2);
      break;
    default:
      gett_tile<2, 2, 2, kP>(it.g, it.A, it.B, it.C, tm * GroupLds0::BM, tn * GroupLds0::BN, kz, lds.t0);
  }
}

template <int kP>
__global__ __launch_bounds__(256) void gett_group_kernel(const GroupItem* __restrict__ items,
                                                         const int* __restrict__ tile_item) {
  group_tile<kP>(items, tile_item);
}

// the same for the Coulomb blocks of a call built together (a symbol of its own in profiles)
template <int kP>
__global__ __launch_bounds__(256) void coulomb_group_kernel(const GroupItem* __restrict__ items,
                                                            const int* __restrict__ tile_item) {
  group_tile<kP>(items, tile_item);
}

// items of the big shape (128 x 128)
template <int kP>
__global__ __launch_bounds__(256) void gett_group_big_kernel(const GroupItem* __restrict__ items,
                                                             const int* __restrict__ tile_item) {
  using Lds = TileLds<4, 4, 2, typename Mfma<kP>::T>;
  __shared__ Lds lds;
  const int b = xcd_tile_windowed(blockIdx.x, gridDim.x);
  const GroupItem& it = items[tile_item[b]];
  const int t = b - it.tile0;
  const int per = it.tiles_m * it.tiles_n;
  const int kz = t / per;
  const int r = t - kz * per;
  const int tm = r / it.tiles_n;
  const int tn = r - tm * it.tiles_n;
  gett_tile<4, 4, 2, kP>(it.g, it.A, it.B, it.C, tm * Lds::BM, tn * Lds::BN, kz, lds);
}

// split-K items: C = alpha * sum_z part[z] (+ C), fixed order of z; the loads of eight
// partial tiles are issued together, the sum runs in z order
__global__ __launch_bounds__(256) void group_reduce_kernel(const GroupItem* __restrict__ items,
                                                           const ReduceBlock* __restrict__ blocks) {
  const ReduceBlock rb = blocks[blockIdx.x];
  const GroupItem& it = items[rb.item];
  const GettDesc& g = it.g;
  const long long mn = (long long)g.M * g.N;
  const long long i = (long long)rb.e0 + threadIdx.x;
  if (i >= mn) return;
  const double* part = g.part + i;
  const int ns = it.splits;
  double s = 0.0;
  int z = 0;
  for (; z + 8 <= ns; z += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(long long)(z + u) * mn];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; z < ns; ++z) s += part[(long long)z * mn];
  const int m = (int)(i / g.N), nn = (int)(i - (long long)m * g.N);
  const long long o = decode_fast(m, g.nm, g.md, g.mmag, g.msh, g.cm) +
                      decode_fast(nn, g.nn, g.nd, g.nmag, g.nsh, g.cn);
  double v = g.alpha * s;
  if (g.beta) v += it.C[o];
  it.C[o] = v;
}

void launch_gett_group(const GroupItem* items, const int* tile_item, int n, int tiles, bool big,
                       int prec, hipStream_t st, bool coulomb) {
  if (n <= 0 || tiles <= 0) return;
  const dim3 grid((unsigned)tiles), block(256);
  if (coulomb && !big) {
    if (prec == 2)
      hipLaunchKernelGGL(coulomb_group_kernel<2>, grid, block, 0, st, items, tile_item);
    else if (prec == 1)
      hipLaunchKernelGGL(coulomb_group_kernel<1>, grid, block, 0, st, items, tile_item);
    else
      hipLaunchKernelGGL(coulomb_group_kernel<0>, grid, block, 0, st, items, tile_item);
    return;
  }
  if (big) {
    if (prec == 2)
      hipLaunchKernelGGL(gett_group_big_kernel<2>, grid, block, 0, st, items, tile_item);
    else if (prec == 1)
      hipLaunchKernelGGL(gett_group_big_kernel<1>, grid, block, 0, st, items, tile_item);
    else
      hipLaunchKernelGGL(gett_group_big_kernel<0>, grid, block, 0, st, items, tile_item);
    return;
  }
  if (prec == 2)
    hipLaunchKernelGGL(gett_group_kernel<2>, grid, block, 0, st, items, tile_item);
  else if (prec == 1)
    hipLaunchKernelGGL(gett_group_kernel<1>, grid, block, 0, st, items, tile_item);
  else
    hipLaunchKernelGGL(gett_group_kernel<0>, grid, block, 0, st, items, tile_item);
}

void launch_group_reduce(const GroupItem* items, const ReduceBlock* blocks, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(group_reduce_kernel, dim3((unsigned)nblocks), dim3(256), 0, st, items, blocks);
}

// ---------------------------------------------------------------------------
// Grouped dot products: block b of the launch adds its share of item i's sum into
// partial[b]; the final weighted sum reads the partials in a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dot_group_kernel(const DotItem* __restrict__ items, int n,
                                                        double* __restrict__ partial) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (items[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const DotItem& it = items[lo];
  const int j = b - it.blk0;
  double sum = 0.0;
  if (it.d.K < (1LL << 31)) {
    // the decode tables copied to registers once (constant indices after unrolling), then
    // four index pairs decoded and loaded before they are summed (same order as one at a time)
    constexpr int NC = 2 * kMaxComp;
    const int nk = it.d.nk;
    unsigned kd[NC], mag[NC];
    int sh[NC];
    long long as[NC], bs[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const bool on = c < nk;
      kd[c] = on ? (unsigned)it.d.kd[c] : 1u;
      mag[c] = on ? it.d.dm.mag[c] : 0u;
      sh[c] = on ? it.d.dm.sh[c] : 0;
      as[c] = on ? it.d.as[c] : 0;
      bs[c] = on ? it.d.bs[c] : 0;
    }
    auto dec = [&](unsigned idx, long long& oa, long long& ob) {
      oa = 0;
      ob = 0;
#pragma unroll
      for (int c = NC - 1; c >= 0; --c) {
        if (c < nk) {
          const unsigned q = (unsigned)(((unsigned long long)idx * mag[c]) >> sh[c]);
          const long long r = (long long)(idx - q * kd[c]);
          oa += r * as[c];
          ob += r * bs[c];
          idx = q;
        }
      }
    };
    const double* __restrict__ A = it.A;
    const double* __restrict__ B = it.B;
    const unsigned K = (unsigned)it.d.K, stride = 256u * (unsigned)it.nblk;
    unsigned i = (unsigned)j * 256u + threadIdx.x;
    for (; i < K && K - i > 3u * stride; i += 4u * stride) {
      double a[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        long long oa, ob;
        dec(i + u * stride, oa, ob);
        a[u] = A[oa];
        bv[u] = B[ob];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) sum += a[u] * bv[u];
    }
    for (; i < K; i += stride) {
      long long oa, ob;
      dec(i, oa, ob);
      sum += A[oa] * B[ob];
    }
  } else {
    for (long long i = j * 256LL + threadIdx.x; i < it.d.K; i += 256LL * it.nblk) {
      long long oa, ob;
      decode2(i, it.d.nk, it.d.kd, it.d.as, it.d.bs, oa, ob);
      sum += it.A[oa] * it.B[ob];
    }
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[b] = red[0];
}

void launch_dot_group(const DotItem* items, int n, int blocks, double* partial, hipStream_t st) {
  if (n <= 0 || blocks <= 0) return;
  hipLaunchKernelGGL(dot_group_kernel, dim3((unsigned)blocks), dim3(256), 0, st, items, n, partial);
}

// ---------------------------------------------------------------------------
// Gather-accumulate into a contiguous output: element x (multi-index) belongs to the
// class given by which sub-space each index falls in; every entry of that class adds
// coef * src[base + sum_k x_k ss_k], in entry order.
// ---------------------------------------------------------------------------
// Each workgroup covers 512 elements of one class (the box of index ranges the class
// stands for, last index fastest; two per lane), so the entry list it walks is the same for
// every lane: entries load through the scalar cache and four entries (eight source values
// per lane) are in flight at a time, summed in entry order.
// tpe > 1 (small outputs, long entry lists): tpe consecutive lanes share an element, lane j
// of the group sums entries j, j + tpe, ... and a fixed butterfly adds the group's partial
// sums (deterministic for a given tpe).
constexpr int kGatherEpl = 2;   // output elements per lane when lanes do not share one
constexpr int kGatherEif = 8 / kGatherEpl;   // entries in flight (eight loads per lane)
// K32: every output and source offset of the launch is below 2^31 (the host checks), so
// the element decode and the source offsets run in 32-bit arithmetic (unsigned, so partial
// sums may wrap: the final offsets are in range).
template <bool K32>
__global__ __launch_bounds__(256) void gather_kernel(const GatherDesc* __restrict__ descs, int nd) {
  using Idx = typename std::conditional<K32, unsigned, long long>::type;
  // output of this workgroup: the last with blk0 <= blockIdx.x
  int dl = 0, dh = nd - 1;
  while (dl < dh) {
    const int mid = (dl + dh + 1) >> 1;
    if (descs[mid].blk0 <= (int)blockIdx.x) dl = mid;
    else dh = mid - 1;
  }
  const GatherDesc& g = descs[dl];
  const GatherEntry* __restrict__ ent = g.ent;
  double* __restrict__ out = g.out;
  const int tpe = g.tpe;
  const int b = (int)blockIdx.x - g.blk0;
  const int ncls = 1 << g.rank;
  int c = 0;
  while (c + 1 < ncls && b >= g.blk[c + 1]) ++c;
  int lo[4] = {0, 0, 0, 0}, len[4] = {1, 1, 1, 1};
  long long cnt = 1;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < g.rank) {
      const bool hi = (c >> k) & 1;
      lo[k] = hi ? g.split[k] : 0;
      len[k] = hi ? g.dim[k] - g.split[k] : g.split[k];
      cnt *= len[k];
    }
  // element e of the class -> its multi-index x and output offset
  auto decode = [&](long long e64, int* x) {
    Idx e = (Idx)e64, o = 0;
#pragma unroll
    for (int k = 3; k >= 0; --k)
      if (k < g.rank) {
        const Idx q = e / (Idx)len[k];
        x[k] = lo[k] + (int)(e - q * (Idx)len[k]);
        e = q;
      }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < g.rank) o = o * (Idx)g.dim[k] + (Idx)x[k];
    return (long long)o;
  };
  auto off = [&](const GatherEntry& en, const int* x) {
    const Idx v = (Idx)en.base + (Idx)x[0] * (Idx)en.ss[0] + (Idx)x[1] * (Idx)en.ss[1] +
                  (Idx)x[2] * (Idx)en.ss[2] + (Idx)x[3] * (Idx)en.ss[3];
    return (long long)v;
  };
  if (tpe == 1) {
    // kGatherEpl elements per lane (e, e + 256, ...): each entry's scalar loads serve all
    const long long e0 = (long long)(b - g.blk[c]) * (256 * kGatherEpl) + threadIdx.x;
    int x[kGatherEpl][4];
    long long o[kGatherEpl];
    bool live[kGatherEpl];
#pragma unroll
    for (int j = 0; j < kGatherEpl; ++j) {
      live[j] = e0 + 256 * j < cnt;
#pragma unroll
      for (int k = 0; k < 4; ++k) x[j][k] = 0;
      o[j] = decode(live[j] ? e0 + 256 * j : e0, x[j]);   // dead slots repeat element e0
    }
    double acc[kGatherEpl];
#pragma unroll
    for (int j = 0; j < kGatherEpl; ++j) acc[j] = 0.0;
    const int end = live[0] ? g.cls[c + 1] : g.cls[c];
    int i = g.cls[c];
    for (; i + kGatherEif - 1 < end; i += kGatherEif) {
      double v[kGatherEif][kGatherEpl];
#pragma unroll
      for (int u = 0; u < kGatherEif; ++u)
#pragma unroll
        for (int j = 0; j < kGatherEpl; ++j) v[u][j] = ent[i + u].src[off(ent[i + u], x[j])];
#pragma unroll
      for (int u = 0; u < kGatherEif; ++u)
#pragma unroll
        for (int j = 0; j < kGatherEpl; ++j) acc[j] = fma(ent[i + u].coef, v[u][j], acc[j]);
    }
    for (; i < end; ++i)
#pragma unroll
      for (int j = 0; j < kGatherEpl; ++j) acc[j] = fma(ent[i].coef, ent[i].src[off(ent[i], x[j])], acc[j]);
#pragma unroll
    for (int j = 0; j < kGatherEpl; ++j)
      if (live[j]) out[o[j]] += acc[j];
    return;
  }
  const int sub = threadIdx.x % tpe;
  const long long e = (long long)(b - g.blk[c]) * (256 / tpe) + threadIdx.x / tpe;
  const bool live = e < cnt;   // whole groups of tpe lanes share e, so shuffles stay in a group
  int x[4] = {0, 0, 0, 0};
  const long long o = decode(e, x);
  double acc = 0.0;
  const int end = live ? g.cls[c + 1] : g.cls[c];
  int i = g.cls[c] + sub;
  for (; i + 3 * tpe < end; i += 4 * tpe) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = ent[i + u * tpe].src[off(ent[i + u * tpe], x)];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(ent[i + u * tpe].coef, v[u], acc);
  }
  for (; i < end; i += tpe) acc = fma(ent[i].coef, ent[i].src[off(ent[i], x)], acc);
  for (int w = tpe >> 1; w > 0; w >>= 1) acc += __shfl_xor(acc, w, 64);
  if (live && sub == 0) out[o] += acc;
}

long long gather_prepare(GatherDesc& g) {
  const int ncls = 1 << g.rank;
  long long total = 0;
  for (int c = 0; c < ncls; ++c) {
    if (g.cls[c + 1] == g.cls[c]) continue;
    long long cnt = 1;
    for (int k = 0; k < g.rank; ++k) cnt *= ((c >> k) & 1) ? g.dim[k] - g.split[k] : g.split[k];
    total += cnt;
  }
  // lanes per element: enough lanes to fill the chip (>= 2^18) for small outputs, at most 64
  int tpe = 1;
  while (tpe < 64 && total * tpe < (1LL << 18)) tpe <<= 1;
  g.tpe = tpe;
  long long blocks = 0;
  for (int c = 0; c < ncls; ++c) {
    g.blk[c] = (int)blocks;
    if (g.cls[c + 1] == g.cls[c]) continue;
    long long cnt = 1;
    for (int k = 0; k < g.rank; ++k) cnt *= ((c >> k) & 1) ? g.dim[k] - g.split[k] : g.split[k];
    blocks += tpe == 1 ? (cnt + 256 * kGatherEpl - 1) / (256 * kGatherEpl) : (cnt * tpe + 255) / 256;
  }
  for (int c = ncls; c <= 16; ++c) g.blk[c] = (int)blocks;
  return blocks;
}

void launch_gather_multi(const GatherDesc* descs, int n, long long blocks, hipStream_t st, bool k32) {
  if (n <= 0 || blocks <= 0) return;
  if (k32)
    hipLaunchKernelGGL(gather_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, descs, n);
  else
    hipLaunchKernelGGL(gather_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, descs, n);
}

// ---------------------------------------------------------------------------
// Deterministic dot product over a strided multi-index
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 512;
int dot_partials() { return kDotBlocks; }

__global__ __launch_bounds__(256) void dot_kernel(DotDesc d, const double* __restrict__ A,
                                                  const double* __restrict__ B,
                                                  double* __restrict__ partial) {
  __shared__ double red[256];
  double sum = 0.0;
  const bool fast = d.K < (1LL << 31);
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < d.K; i += 256LL * gridDim.x) {
    long long oa, ob;
    if (fast) decode2_fast<2 * kMaxComp>((unsigned)i, d.nk, d.kd, d.dm, d.as, d.bs, oa, ob);
    else decode2(i, d.nk, d.kd, d.as, d.bs, oa, ob);
    sum += A[oa] * B[ob];
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial, int n,
                                                           double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

void div_magic(const int* d, int n, DivMagic& m) {
  for (int c = 0; c < 2 * kMaxComp; ++c) {
    unsigned mg;
    int sh;
    magic_of(c < n ? std::max(1, d[c]) : 1, mg, sh);
    m.mag[c] = mg;
    m.sh[c] = sh;
  }
}

void launch_dot(const DotDesc& d0, const double* A, const double* B, double* partial, double* out,
                hipStream_t st) {
  DotDesc d = d0;
  div_magic(d.kd, d.nk, d.dm);
  hipLaunchKernelGGL(dot_kernel, dim3(kDotBlocks), dim3(256), 0, st, d, A, B, partial);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, partial, kDotBlocks, out);
}

// ---------------------------------------------------------------------------
// Packed copy of a strided view
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(PackDesc d, const double* __restrict__ src,
                                                   double* __restrict__ dst) {
  const bool fast = d.n < (1LL << 31);
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < d.n; e += 256LL * gridDim.x) {
    long long off = 0, unused;
    if (fast) {
      decode2_fast<2 * kMaxComp>((unsigned)e, d.rank, d.d, d.dm, d.ss, nullptr, off, unused);
    } else {
      long long idx = e;
      for (int c = d.rank - 1; c >= 0; --c) {
        const long long q = idx / d.d[c];
        off += (idx - q * d.d[c]) * d.ss[c];
        idx = q;
      }
    }
    dst[e] = src[off];
  }
}

// Transposing packs: the source's unit-stride dimension u is not the target's last one w.
// A workgroup copies a 32 x 32 tile of (u, w) for one index of the other dimensions through
// LDS, reading along u and writing along w, so both sides move whole cache lines.
struct PackTile {
  int nr = 0;                            // other dimensions
  int rd[2 * kMaxComp] = {};             // their extents (row-major)
  long long rs[2 * kMaxComp] = {}, ro[2 * kMaxComp] = {};   // their source and target strides
  int du = 1, dw = 1;
  long long su = 1, ou = 0, sw = 0, ow = 1;
  long long rest = 1;                    // product of rd
};
__global__ __launch_bounds__(256) void pack_tiled_kernel(PackTile t, const double* __restrict__ src,
                                                         double* __restrict__ dst) {
  __shared__ double T[32][33];
  const int tu = (t.du + 31) / 32, tw = (t.dw + 31) / 32;
  const long long work = t.rest * tu * tw;
  for (long long w = blockIdx.x; w < work; w += gridDim.x) {
    long long r = w / (tu * tw);
    const int q = (int)(w - r * (tu * tw));
    const int u0 = (q % tu) * 32, w0 = (q / tu) * 32;
    long long sb = 0, ob = 0;
    for (int c = t.nr - 1; c >= 0; --c) {
      const long long x = r % t.rd[c];
      r /= t.rd[c];
      sb += x * t.rs[c];
      ob += x * t.ro[c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int b = e & 31, a = e >> 5;   // b along u (unit stride in the source)
      const int uu = u0 + b, ww = w0 + a;
      if (uu < t.du && ww < t.dw) T[a][b] = src[sb + uu * t.su + ww * t.sw];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int a = e & 31, b = e >> 5;   // a along w (unit stride in the target)
      const int uu = u0 + b, ww = w0 + a;
      if (uu < t.du && ww < t.dw) dst[ob + uu * t.ou + ww * t.ow] = T[a][b];
    }
  }
}

void launch_pack(const PackDesc& d0, const double* src, double* dst, hipStream_t st) {
  if (d0.n <= 0) return;
  // the target is contiguous in the order of the dimensions (the last fastest)
  long long os[2 * kMaxComp];
  {
    long long m = 1;
    for (int k = d0.rank - 1; k >= 0; --k) {
      os[k] = m;
      m *= d0.d[k];
    }
  }
  const int w = d0.rank - 1;
  int u = -1;
  for (int k = 0; k < d0.rank; ++k)
    if (d0.ss[k] == 1 && d0.d[k] > 1) u = k;
  if (u >= 0 && u != w && d0.d[u] >= 8 && d0.d[w] >= 8) {
    PackTile t;
    for (int k = 0; k < d0.rank; ++k) {
      if (k == u || k == w) continue;
      t.rd[t.nr] = d0.d[k];
      t.rs[t.nr] = d0.ss[k];
      t.ro[t.nr] = os[k];
      t.rest *= d0.d[k];
      ++t.nr;
    }
    t.du = d0.d[u]; t.su = d0.ss[u]; t.ou = os[u];
    t.dw = d0.d[w]; t.sw = d0.ss[w]; t.ow = os[w];
    const long long work = t.rest * ((t.du + 31) / 32) * ((t.dw + 31) / 32);
    const unsigned grid = (unsigned)std::min<long long>(work, 1LL << 20);
    hipLaunchKernelGGL(pack_tiled_kernel, dim3(grid), dim3(256), 0, st, t, src, dst);
    return;
  }
  PackDesc d = d0;
  div_magic(d.d, d.rank, d.dm);
  const long long blocks = std::min<long long>((d.n + 255) / 256, 16384);
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d, src, dst);
}

// ---------------------------------------------------------------------------
// Pair antisymmetriser of a pre-image added into a [P][P][H][H] tensor
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void antisym_add_kernel(const double* __restrict__ X, double* __restrict__ O,
                                                          int nP, int nH, long long total) {
  const long long hh = (long long)nH * nH, qs = hh, ps = (long long)nP * hh;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const long long p = e / ps, r1 = e - p * ps;
    const long long q = r1 / qs, r2 = r1 - q * qs;
    const long long i = r2 / nH, j = r2 - i * nH;
    const long long qp = q * ps + p * qs;
    O[e] += X[e] - X[qp + r2] - X[p * ps + q * qs + j * nH + i] + X[qp + j * nH + i];
  }
}

void launch_antisym_add(const double* X, double* O, int nP, int nH, hipStream_t st) {
  const long long total = (long long)nP * nP * nH * nH;
  if (total <= 0) return;
  const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>((total + 255) / 256, 16384));
  hipLaunchKernelGGL(antisym_add_kernel, dim3(grid), dim3(256), 0, st, X, O, nP, nH, total);
}

// Pair blockIdx.y of the list; 32-bit index arithmetic (the launcher checks the size).
__global__ __launch_bounds__(256) void antisym_add_list_kernel(AntisymList l, int nP, int nH, unsigned total) {
  const double* __restrict__ X = l.X[blockIdx.y];
  double* __restrict__ O = l.O[blockIdx.y];
  const unsigned hh = (unsigned)nH * nH, ps = (unsigned)nP * hh;
  for (unsigned e = blockIdx.x * 256u + threadIdx.x; e < total; e += 256u * gridDim.x) {
    const unsigned p = e / ps, r1 = e - p * ps;
    const unsigned q = r1 / hh, r2 = r1 - q * hh;
    const unsigned i = r2 / nH, j = r2 - i * nH;
    const unsigned qp = q * ps + p * hh;
    O[e] += X[e] - X[qp + r2] - X[p * ps + q * hh + j * nH + i] + X[qp + j * nH + i];
  }
}

void launch_antisym_add_list(const AntisymList& l, int nP, int nH, hipStream_t st) {
  const long long total = (long long)nP * nP * nH * nH;
  if (total <= 0 || l.n <= 0) return;
  if (total >= (1LL << 31)) {
    for (int k = 0; k < l.n; ++k) launch_antisym_add(l.X[k], l.O[k], nP, nH, st);
    return;
  }
  const unsigned gx = (unsigned)std::max<long long>(1, std::min<long long>((total + 255) / 256, 16384));
  hipLaunchKernelGGL(antisym_add_list_kernel, dim3(gx, (unsigned)l.n), dim3(256), 0, st, l, nP, nH,
                     (unsigned)total);
}

// ---------------------------------------------------------------------------
// Same-spin ladder on unique pairs: packing of the antisymmetrised integrals and of the
// amplitudes, and the antisymmetric fill of the result
// ---------------------------------------------------------------------------
// One workgroup per (row, pair of 32-wide tiles X <= Y of the x and y ranges): the tile
// M[X][Y] of M[x][y] = jb[p - b0][x][q - qoff][y] and its mirror M[Y][X] are read with y
// fastest into LDS, and V is written in packed order (y fastest inside each x).
constexpr int kPackTile = 32;
constexpr int kPackRun = 16;   // rows per run of the resident-block packs (one 128-byte line of q)

// position of the particle pair (a, b) among the pairs a <= b in a-major order
__device__ __forceinline__ long long pair_pos(int nP, int a, int b) {
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
  const long long al = a;
  return al * nP - al * (al - 1) / 2 + (b - a);
}

// Integral source of the packs: a batch jb[p - b0][x][q - qoff][y] = (p x|q y) (kFull =
// false) or the resident packed block K[pair(p, x)][pair(q, y)] (kFull = true).
template <bool kFull>
__global__ __launch_bounds__(256) void ladder_pack_v_kernel(const double* __restrict__ jb, int nP, int b0,
                                                            int qoff, int nq,
                                                            const LadderPair* __restrict__ rowtab, int rows,
                                                            int ntp, int sym, long long kpx,
                                                            double* __restrict__ Vp, double* __restrict__ Va,
                                                            long long m0) {
  __shared__ double A[kPackTile][kPackTile + 1], Bm[kPackTile][kPackTile + 1];
  const int nT = (nP + kPackTile - 1) / kPackTile;
  const long long sq = nP, sx = (long long)nq * nP, sp = sx * nP;
  const long long npk = (long long)nP * (nP + 1) / 2;
  const long long work = (long long)rows * ntp;
  for (long long w = blockIdx.x; w < work; w += gridDim.x) {
    // work order: runs of kPackRun consecutive rows (one p, consecutive q in the row table)
    // with the rows fastest for each tile pair, the runs of one XCD contiguous when one
    // pass of the grid covers the work.  The reads with x < p and y < q (K[pair(x, p)]
    // [pair(y, q)], one element per cache line for a single row) are contiguous along q, so
    // the run's workgroups, resident on one XCD at the same time, share those lines in L2.
    const long long L = gridDim.x == work ? xcd_tile((int)w, (int)work) : w;
    const long long run = L / ((long long)kPackRun * ntp);
    const long long rem = L - run * kPackRun * ntp;
    const int rr = (int)min((long long)kPackRun, rows - run * kPackRun);
    int t = (int)(rem / rr);
    const int row = (int)(run * kPackRun + (rem - (long long)t * rr));
    // tile pair t -> (tx, ty), tx <= ty, tx-major
    int tx = 0;
    while (t >= nT - tx) {
      t -= nT - tx;
      ++tx;
    }
    const int ty = tx + t;
    const LadderPair pq = rowtab[row];
    const int p = pq.a, q = pq.b;
    const int X0 = tx * kPackTile, Y0 = ty * kPackTile;
    __syncthreads();
    if constexpr (!kFull) {
      const double* M = jb + (p - b0) * sp + (long long)(q - qoff) * sq;
      for (int e = threadIdx.x; e < kPackTile * kPackTile; e += 256) {
        const int i = e / kPackTile, j = e % kPackTile;
        const int x = X0 + i, y = Y0 + j;
        A[i][j] = (x < nP && y < nP) ? M[x * sx + y] : 0.0;
        const int x2 = Y0 + i, y2 = X0 + j;
        Bm[i][j] = (x2 < nP && y2 < nP) ? M[x2 * sx + y2] : 0.0;
      }
    } else {
      // (p x|q y) from the symmetric K, read where consecutive lanes meet consecutive
      // columns: row pair(p, x) along y while y >= q (columns pair(q, y) are contiguous),
      // row pair(y, q) along x while y < q and x >= p (columns pair(p, x) contiguous, by the
      // symmetry of K); the rest (x < p, y < q) element by element.  Pass 0 walks y
      // fastest, pass 1 x.
      auto J = [&](int x, int y) -> double {
        if (y >= q) return jb[pair_pos(nP, p, x) * npk + pair_pos(nP, q, y)];
        if (x >= p) return jb[pair_pos(nP, y, q) * npk + pair_pos(nP, p, x)];
        return jb[pair_pos(nP, x, p) * npk + pair_pos(nP, y, q)];
      };
      // tile T (0: A holds S[X0 + i][Y0 + j]; 1: Bm holds S[Y0 + i][X0 + j]) over S[x][y] =
      // (p x|q y)
      for (int e = threadIdx.x; e < kPackTile * kPackTile; e += 256) {
        const int i = e / kPackTile, j = e % kPackTile;   // j fastest
        {
          const int x = X0 + i, y = Y0 + j;
          const bool in = x < nP && y < nP;
          if (!in) A[i][j] = 0.0;
          else if (y >= q || x < p) A[i][j] = J(x, y);
        }
        {
          const int x = Y0 + i, y = X0 + j;
          const bool in = x < nP && y < nP;
          if (!in) Bm[i][j] = 0.0;
          else if (y >= q || x < p) Bm[i][j] = J(x, y);
        }
      }
      for (int e = threadIdx.x; e < kPackTile * kPackTile; e += 256) {
        const int i = e % kPackTile, j = e / kPackTile;   // i fastest
        {
          const int x = X0 + i, y = Y0 + j;
          if (x < nP && y < nP && y < q && x >= p) A[i][j] = J(x, y);
        }
        {
          const int x = Y0 + i, y = X0 + j;
          if (x < nP && y < nP && y < q && x >= p) Bm[i][j] = J(x, y);
        }
      }
    }
    __syncthreads();
    double* out = Vp + (long long)row * kpx;
    // strict pairs' antisymmetric row in the same pass (sym mode with Va)
    double* outa = (Va && pq.m >= 0) ? Va + (pq.m - m0) * ((long long)nP * (nP - 1) / 2) : nullptr;
    for (int e = threadIdx.x; e < kPackTile * kPackTile; e += 256) {
      const int i = e / kPackTile, j = e % kPackTile;
      const int x = X0 + i, y = Y0 + j;
      if (x >= nP || y >= nP || (sym ? y < x : y <= x)) continue;
      const double u = A[i][j], v = Bm[j][i];   // (p x|q y), (p y|q x)
      const long long xl = x;
      const long long ka = xl * nP - xl * (xl + 1) / 2 + (y - x - 1);
      const long long k = sym ? xl * nP - xl * (xl - 1) / 2 + (y - x) : ka;
      out[k] = sym ? (x == y ? u : u + v) : u - v;
      if (outa && y > x) outa[ka] = u - v;
    }
  }
}

// Bp[Q][pair(a, b)] = B[Q][off + a][off + b] over the pairs a <= b of nP orbitals from off
__global__ __launch_bounds__(256) void pack_pairs_kernel(const double* __restrict__ B, int N, int off, int nP,
                                                         long long total, double* __restrict__ Bp) {
  const long long npk = (long long)nP * (nP + 1) / 2;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long Q = e / ((long long)nP * nP);
    const int r = (int)(e - Q * nP * nP);
    const int a = r / nP, b = r - a * nP;
    if (a > b) continue;
    Bp[Q * npk + pair_pos(nP, a, b)] = B[(Q * N + off + a) * N + off + b];
  }
}

// K[i][j] = K[j][i] for the elements whose row block i / blk lies below the column block
// j / blk (those a triangular contraction with tri = blk leaves unwritten), through LDS.
// Work item w is a run of G 32 x 32 tiles (ti, tj0 .. tj0 + G - 1) of the lower part, taken
// from the transposed upper tiles; only lower tiles are enumerated: row ti of tiles holds
// (ti / per) (per / G) items (per = blk / 32, a multiple of G), so the items before row ti
// number cum(ti) = (per / G) (per Q (Q - 1) / 2 + S Q) with Q = ti / per, S = ti % per, and
// the row of w is the last ti with cum(ti) <= w.
template <int G>
__global__ __launch_bounds__(256) void mirror_lower_kernel(double* __restrict__ K, long long n, int blk) {
  __shared__ double T[G][32][33];
  const long long nt = (n + 31) / 32;
  const long long per = blk / 32, cpg = per / G;
  auto cum = [&](long long t) -> long long {
    const long long Q = t / per, S = t - Q * per;
    return cpg * (per * Q * (Q - 1) / 2 + S * Q);
  };
  const long long total = cum(nt);
  for (long long w = blockIdx.x; w < total; w += gridDim.x) {
    long long lo = 0, hi = nt - 1;
    while (lo < hi) {
      const long long mid = (lo + hi + 1) / 2;
      if (cum(mid) <= w) lo = mid;
      else hi = mid - 1;
    }
    const long long ti = lo, tj0 = (w - cum(ti)) * G;
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g)
      for (int e = threadIdx.x; e < 1024; e += 256) {
        const int a = e / 32, b = e % 32;
        const long long r = (tj0 + g) * 32 + a, c = ti * 32 + b;   // source: upper tile (tj, ti)
        T[g][a][b] = (r < n && c < n) ? K[r * n + c] : 0.0;
      }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g)
      for (int e = threadIdx.x; e < 1024; e += 256) {
        const int a = e / 32, b = e % 32;
        const long long r = ti * 32 + a, c = (tj0 + g) * 32 + b;
        if (r < n && c < n) K[r * n + c] = T[g][b][a];
      }
  }
}

static unsigned grid_for(long long n);

void launch_pack_pairs(const double* B, int N, int off, int nP, int M, double* Bp, hipStream_t st) {
  const long long total = (long long)M * nP * nP;
  if (total <= 0) return;
  hipLaunchKernelGGL(pack_pairs_kernel, dim3(grid_for(total)), dim3(256), 0, st, B, N, off, nP, total, Bp);
}

void launch_mirror_lower(double* K, long long n, int blk, hipStream_t st) {
  const long long nt = (n + 31) / 32;
  if (nt <= 1 || blk % 32 != 0) return;
  // items of four tiles when a block holds a multiple of four tiles (one per tile else)
  const long long per = blk / 32, Q = nt / per, S = nt - Q * per;
  const int G = per % 4 == 0 ? 4 : 1;
  const long long items = per / G * (per * Q * (Q - 1) / 2 + S * Q);
  if (items <= 0) return;
  const unsigned grid = (unsigned)std::min<long long>(items, 1LL << 20);
  if (G == 4)
    hipLaunchKernelGGL(mirror_lower_kernel<4>, dim3(grid), dim3(256), 0, st, K, n, blk);
  else
    hipLaunchKernelGGL(mirror_lower_kernel<1>, dim3(grid), dim3(256), 0, st, K, n, blk);
}

__global__ __launch_bounds__(256) void ladder_pack_t_kernel(const double* __restrict__ T, int nP, int nH,
                                                            const LadderPair* __restrict__ ktab, int kp,
                                                            const LadderPair* __restrict__ ntab, int np,
                                                            int mode, double* __restrict__ Tp) {
  const long long total = (long long)kp * np;
  const long long hh = (long long)nH * nH;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const int n = (int)(e / kp), k = (int)(e - (long long)n * kp);
    const LadderPair xy = ktab[k], ij = ntab[n];
    const long long h = (long long)ij.a * nH + ij.b;
    const double u = T[((long long)xy.a * nP + xy.b) * hh + h];
    if (mode == 0) {
      Tp[e] = u;
    } else {
      const double w = T[((long long)xy.b * nP + xy.a) * hh + h];
      Tp[e] = mode == 1 ? 0.5 * (u + w) : 0.5 * (u - w);
    }
  }
}

__global__ __launch_bounds__(256) void ladder_unpack_anti_kernel(const double* __restrict__ Xp, int rows, int np,
                                                                 int ldx, const LadderPair* __restrict__ rowtab,
                                                                 const LadderPair* __restrict__ ntab, int nP,
                                                                 int nH, double c, double* __restrict__ O) {
  const long long total = (long long)rows * np;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const int row = (int)(e / np), n = (int)(e - (long long)row * np);
    const LadderPair pq = rowtab[row], ij = ntab[n];
    const long long p = pq.a, q = pq.b;
    const double v = c * Xp[(long long)row * ldx + n];
    O[((p * nP + q) * nH + ij.a) * nH + ij.b] += v;
    O[((q * nP + p) * nH + ij.a) * nH + ij.b] -= v;
    O[((p * nP + q) * nH + ij.b) * nH + ij.a] -= v;
    O[((q * nP + p) * nH + ij.b) * nH + ij.a] += v;
  }
}

__global__ __launch_bounds__(256) void ladder_unpack_sym_kernel(const double* __restrict__ Xs,
                                                                const double* __restrict__ Xa, int rows, int np,
                                                                int npa, int m0,
                                                                const LadderPair* __restrict__ rowtab,
                                                                const LadderPair* __restrict__ ntab, int nP,
                                                                int nH, double c, double* __restrict__ O) {
  const long long total = (long long)rows * np;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const int row = (int)(e / np), n = (int)(e - (long long)row * np);
    const LadderPair pq = rowtab[row], ij = ntab[n];
    const double S = Xs[e];
    const double A = (pq.m >= 0 && ij.m >= 0) ? Xa[(long long)(pq.m - m0) * npa + ij.m] : 0.0;
    const long long p = pq.a, q = pq.b;
    O[((p * nP + q) * nH + ij.a) * nH + ij.b] += c * (S + A);
    if (ij.a != ij.b) O[((p * nP + q) * nH + ij.b) * nH + ij.a] += c * (S - A);
    if (p != q) {
      O[((q * nP + p) * nH + ij.a) * nH + ij.b] += c * (S - A);
      if (ij.a != ij.b) O[((q * nP + p) * nH + ij.b) * nH + ij.a] += c * (S + A);
    }
  }
}

static unsigned grid_for(long long n) {
  return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 16384));
}

void launch_ladder_pack_v(const double* jb, int nP, int b0, int qoff, int nq, const LadderPair* rowtab,
                          int rows, int sym, double* Vp, hipStream_t st, double* Va, long long m0) {
  const long long kpx = sym ? (long long)nP * (nP + 1) / 2 : (long long)nP * (nP - 1) / 2;
  if (rows <= 0 || kpx <= 0) return;
  const int nT = (nP + kPackTile - 1) / kPackTile, ntp = nT * (nT + 1) / 2;
  const long long work = (long long)rows * ntp;
  const unsigned grid = (unsigned)std::min<long long>(work, 1LL << 20);
  hipLaunchKernelGGL(ladder_pack_v_kernel<false>, dim3(grid), dim3(256), 0, st, jb, nP, b0, qoff, nq, rowtab, rows,
                     ntp, sym, kpx, Vp, sym ? Va : nullptr, m0);
}

void launch_ladder_pack_vk(const double* K, int nP, const LadderPair* rowtab, int rows, int sym, double* Vp,
                           hipStream_t st, double* Va, long long m0) {
  const long long kpx = sym ? (long long)nP * (nP + 1) / 2 : (long long)nP * (nP - 1) / 2;
  if (rows <= 0 || kpx <= 0) return;
  const int nT = (nP + kPackTile - 1) / kPackTile, ntp = nT * (nT + 1) / 2;
  const long long work = (long long)rows * ntp;
  const unsigned grid = (unsigned)std::min<long long>(work, 1LL << 20);
  hipLaunchKernelGGL(ladder_pack_v_kernel<true>, dim3(grid), dim3(256), 0, st, K, nP, 0, 0, nP, rowtab, rows, ntp,
                     sym, kpx, Vp, sym ? Va : nullptr, m0);
}

void launch_ladder_pack_t(const double* T, int nP, int nH, const LadderPair* ktab, int kp,
                          const LadderPair* ntab, int np, int mode, double* Tp, hipStream_t st) {
  if (kp <= 0 || np <= 0) return;
  hipLaunchKernelGGL(ladder_pack_t_kernel, dim3(grid_for((long long)kp * np)), dim3(256), 0, st, T, nP, nH,
                     ktab, kp, ntab, np, mode, Tp);
}

void launch_ladder_unpack_anti(const double* Xp, int rows, int np, int ldx, const LadderPair* rowtab,
                               const LadderPair* ntab, int nP, int nH, double c, double* O,
                               hipStream_t st) {
  if (rows <= 0 || np <= 0) return;
  hipLaunchKernelGGL(ladder_unpack_anti_kernel, dim3(grid_for((long long)rows * np)), dim3(256), 0, st, Xp,
                     rows, np, ldx, rowtab, ntab, nP, nH, c, O);
}

void launch_ladder_unpack_sym(const double* Xs, const double* Xa, int rows, int np, int npa, int m0,
                              const LadderPair* rowtab, const LadderPair* ntab, int nP, int nH, double c,
                              double* O, hipStream_t st) {
  if (rows <= 0 || np <= 0) return;
  hipLaunchKernelGGL(ladder_unpack_sym_kernel, dim3(grid_for((long long)rows * np)), dim3(256), 0, st, Xs, Xa,
                     rows, np, npa, m0, rowtab, ntab, nP, nH, c, O);
}

// ---------------------------------------------------------------------------
// Scatter-add with permutation
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void scatter_kernel(ScatterDesc d, const double* __restrict__ src,
                                                      double* __restrict__ out) {
  const bool fast = d.n < (1LL << 31);
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < d.n; i += 256LL * gridDim.x) {
    long long os, oo;
    if (fast) decode2_fast<kMaxComp>((unsigned)i, d.rank, d.d, d.dm, d.ss, d.so, os, oo);
    else decode2(i, d.rank, d.d, d.ss, d.so, os, oo);
    out[oo] += d.coef * src[os];
  }
}

// Transposing variant for a source whose fastest dimension u differs from the target's
// fastest dimension w: a workgroup takes a 32 x 32 tile of (u, w) at one index of the other
// dimensions (ru: their row-major composition, up to kMaxComp - 2 of them), reads it along
// u and writes it along w, both coalesced.  Same arithmetic as scatter_kernel per element.
struct ScatterTile {
  int nr = 0;                  // other dimensions
  int rd[kMaxComp] = {};       // their extents (row-major)
  long long rs[kMaxComp] = {}, ro[kMaxComp] = {};   // their source and target strides
  int du = 1, dw = 1;
  long long su = 0, ou = 0, sw = 0, ow = 0;        // strides of u and w (source, target)
  long long rest = 1;          // product of rd
  double coef = 1.0;
};
__global__ __launch_bounds__(256) void scatter_tiled_kernel(ScatterTile t, const double* __restrict__ src,
                                                            double* __restrict__ out) {
  __shared__ double T[32][33];
  const int tu = (t.du + 31) / 32, tw = (t.dw + 31) / 32;
  const long long work = t.rest * tu * tw;
  for (long long w = blockIdx.x; w < work; w += gridDim.x) {
    long long r = w / (tu * tw);
    const int q = (int)(w - r * (tu * tw));
    const int u0 = (q % tu) * 32, w0 = (q / tu) * 32;
    long long sb = 0, ob = 0;
    for (int c = t.nr - 1; c >= 0; --c) {
      const long long x = r % t.rd[c];
      r /= t.rd[c];
      sb += x * t.rs[c];
      ob += x * t.ro[c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int b = e & 31, a = e >> 5;   // b along u (fastest in the source)
      const int uu = u0 + b, ww = w0 + a;
      T[a][b] = (uu < t.du && ww < t.dw) ? src[sb + uu * t.su + ww * t.sw] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int a = e & 31, b = e >> 5;   // a along w (fastest in the target)
      const int uu = u0 + b, ww = w0 + a;
      if (uu < t.du && ww < t.dw) out[ob + uu * t.ou + ww * t.ow] += t.coef * T[a][b];
    }
  }
}

void launch_scatter(const ScatterDesc& d0, const double* src, double* out, hipStream_t st) {
  if (d0.n <= 0) return;
  // the fastest dimension of the source and of the target
  int u = 0, w = 0;
  for (int k = 1; k < d0.rank; ++k) {
    if (std::llabs(d0.ss[k]) < std::llabs(d0.ss[u])) u = k;
    if (std::llabs(d0.so[k]) < std::llabs(d0.so[w])) w = k;
  }
  if (u != w && d0.d[u] >= 8 && d0.d[w] >= 8 && d0.ss[u] == 1 && d0.so[w] == 1) {
    ScatterTile t;
    for (int k = 0; k < d0.rank; ++k) {
      if (k == u || k == w) continue;
      t.rd[t.nr] = d0.d[k];
      t.rs[t.nr] = d0.ss[k];
      t.ro[t.nr] = d0.so[k];
      t.rest *= d0.d[k];
      ++t.nr;
    }
    t.du = d0.d[u]; t.su = d0.ss[u]; t.ou = d0.so[u];
    t.dw = d0.d[w]; t.sw = d0.ss[w]; t.ow = d0.so[w];
    t.coef = d0.coef;
    const long long work = t.rest * ((t.du + 31) / 32) * ((t.dw + 31) / 32);
    const unsigned grid = (unsigned)std::min<long long>(work, 1LL << 20);
    hipLaunchKernelGGL(scatter_tiled_kernel, dim3(grid), dim3(256), 0, st, t, src, out);
    return;
  }
  ScatterDesc d = d0;
  div_magic(d.d, d.rank, d.dm);
  long long blocks = (d.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d, src, out);
}

// ---------------------------------------------------------------------------
// Reference densities: spin blocks -> spin-orbital tensors over the 2 nA active spin
// orbitals [alpha | beta]; other spin patterns follow from the canonical (alpha-first)
// block by permuting upper and lower indices with the parity sign.
// ---------------------------------------------------------------------------
// Workgroup row blockIdx.x is one upper (creation) tuple, so its spins and block offset are
// uniform; threads take the lower tuples.  The parity of the stable alpha-first sort of a
// tuple is its number of (beta, alpha) pairs in that order.  Row and column indices fit
// 32 bits: (2 nA)^3 <= 2^15 for nA <= 16 (larger active spaces are rejected).
template <int R>
__device__ __forceinline__ void expand_rdm_row(int nA, const double* __restrict__ blocks, double* __restrict__ so,
                                               int row, int l) {
  const int n2 = 2 * nA;
  int nt = 1, bsz = 1;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    nt *= n2;
    bsz *= nA * nA;
  }
  if (l >= nt) return;
  int su[R], pu[R], sl[R], pl[R];
  int tu = row, tl = l;
#pragma unroll
  for (int c = R - 1; c >= 0; --c) {
    const int xu = tu % n2, xl = tl % n2;
    tu /= n2;
    tl /= n2;
    su[c] = xu >= nA;
    pu[c] = xu - su[c] * nA;
    sl[c] = xl >= nA;
    pl[c] = xl - sl[c] * nA;
  }
  int nbu = 0, nbl = 0, par = 0;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    nbu += su[c];
    nbl += sl[c];
  }
  const long long o = (long long)row * nt + l;
  if (nbu != nbl) {
    so[o] = 0.0;
    return;
  }
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = a + 1; b < R; ++b) par += (su[a] > su[b]) + (sl[a] > sl[b]);
  int off = 0;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (su[c] == sp) off = off * nA + pu[c];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (sl[c] == sp) off = off * nA + pl[c];
  const double v = blocks[(long long)nbu * bsz + off];
  so[o] = (par & 1) ? -v : v;
}

template <int R>
__global__ void expand_rdm_kernel(int nA, const double* __restrict__ blocks, double* __restrict__ so) {
  expand_rdm_row<R>(nA, blocks, so, blockIdx.x, blockIdx.y * blockDim.x + threadIdx.x);
}

// gamma1 and gamma2 in one launch: rows [0, 2 nA) are gamma1's, the next (2 nA)^2 gamma2's
// (a row has at most (2 nA)^2 <= 1024 lower tuples, taken 256 at a time)
__global__ void expand_rdm12_kernel(int nA, const double* __restrict__ g1, double* __restrict__ G1,
                                    const double* __restrict__ g2, double* __restrict__ G2) {
  const int n2 = 2 * nA;
  if ((int)blockIdx.x < n2) {
    expand_rdm_row<1>(nA, g1, G1, blockIdx.x, threadIdx.x);
    return;
  }
  for (int l = threadIdx.x; l < n2 * n2; l += blockDim.x) expand_rdm_row<2>(nA, g2, G2, blockIdx.x - n2, l);
}

void launch_expand_rdm12(int nA, const double* g1, double* G1, const double* g2, double* G2, hipStream_t st) {
  const int n2 = 2 * nA;
  if (n2 == 0) return;
  hipLaunchKernelGGL(expand_rdm12_kernel, dim3((unsigned)(n2 + n2 * n2)), dim3(256), 0, st, nA, g1, G1, g2, G2);
}

void launch_expand_rdm(int nA, int rank, const double* blocks, double* so, hipStream_t st) {
  int nt = 1;
  for (int c = 0; c < rank; ++c) nt *= 2 * nA;
  if (nt == 0) return;
  const dim3 grid((unsigned)nt, (unsigned)((nt + 255) / 256));
  if (rank == 1)
    hipLaunchKernelGGL(expand_rdm_kernel<1>, grid, dim3(256), 0, st, nA, blocks, so);
  else if (rank == 2)
    hipLaunchKernelGGL(expand_rdm_kernel<2>, grid, dim3(256), 0, st, nA, blocks, so);
  else
    hipLaunchKernelGGL(expand_rdm_kernel<3>, grid, dim3(256), 0, st, nA, blocks, so);
}

// lambda2[p,q,r,s] = G2 - (g_pr g_qs - g_ps g_qr);  C-convention over spin orbitals.
// (the first n^2 threads also write eta = 1 - gamma1)
__global__ void cumulant2_kernel(int n, const double* __restrict__ G1, const double* __restrict__ G2,
                                 double* __restrict__ L2, double* __restrict__ eta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = n * n * n * n;
  if (i < n * n) eta[i] = ((i / n) == (i % n) ? 1.0 : 0.0) - G1[i];
  if (i >= total) return;
  const int s = i % n, r = (i / n) % n, q = (i / n / n) % n, p = i / n / n / n;
  L2[i] = G2[i] - (G1[p * n + r] * G1[q * n + s] - G1[p * n + s] * G1[q * n + r]);
}

// lambda3 = G3 - det(g g g) - sum_{ij} (-1)^(i+j) g[P_i, S_j] lambda2[P\i, S\j]
// Workgroup row blockIdx.x is the upper triple P (uniform), threads take the lower triples S;
// the three rows g[P_a][*] and the three slices lambda2[P\a][*][*] the row needs are staged
// in LDS first (n = 2 nA <= 32).  G3[P][S] is read from the spin blocks g3 the way
// expand_rdm_kernel<3> forms it (alpha-first block, parity sign, zero unless the numbers of
// beta indices above and below agree), so the spin-orbital G3 is never stored.
__global__ __launch_bounds__(256) void cumulant3_kernel(int n, const double* __restrict__ G1,
                                                        const double* __restrict__ L2,
                                                        const double* __restrict__ g3,
                                                        double* __restrict__ L3) {
  __shared__ double gs[3][32], ls[3][32 * 32];
  const int n2 = n * n, n3 = n2 * n;
  const int u = blockIdx.x;
  const int P[3] = {u / n2, (u / n) % n, u % n};
  // P without its a-th member, in order
  const int U0[3] = {P[1], P[0], P[0]}, U1[3] = {P[2], P[2], P[1]};
  for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) {
    const int a = t / n, c = t - a * n;
    gs[a][c] = G1[P[a] * n + c];
  }
  for (int t = threadIdx.x; t < 3 * n2; t += blockDim.x) {
    const int a = t / n2, c = t - a * n2;
    ls[a][c] = L2[(long long)(U0[a] * n + U1[a]) * n2 + c];
  }
  __syncthreads();
  const int l = blockIdx.y * blockDim.x + threadIdx.x;
  if (l >= n3) return;
  const int S[3] = {l / n2, (l / n) % n, l % n};
  const long long i = (long long)u * n3 + l;
  double g[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) g[a][b] = gs[a][S[b]];
  // determinant part
  const double det = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1])
                   - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0])
                   + g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
  // S without its b-th member, in order
  const int V0[3] = {S[1], S[0], S[0]}, V1[3] = {S[2], S[2], S[1]};
  double gl = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double sgn = ((a + b) & 1) ? -1.0 : 1.0;
      gl += sgn * g[a][b] * ls[a][V0[b] * n + V1[b]];
    }
  // G3[P][S] from the spin blocks
  const int nA = n / 2;
  int su[3], pu[3], sl[3], pl[3], nbu = 0, nbl = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    su[c] = P[c] >= nA;
    pu[c] = P[c] - su[c] * nA;
    sl[c] = S[c] >= nA;
    pl[c] = S[c] - sl[c] * nA;
    nbu += su[c];
    nbl += sl[c];
  }
  double g3v = 0.0;
  if (nbu == nbl) {
    int par = 0, off = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a + 1; b < 3; ++b) par += (su[a] > su[b]) + (sl[a] > sl[b]);
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (su[c] == sp) off = off * nA + pu[c];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (sl[c] == sp) off = off * nA + pl[c];
    const long long bsz = (long long)nA * nA * nA * nA * nA * nA;
    const double v = g3[nbu * bsz + off];
    g3v = (par & 1) ? -v : v;
  }
  L3[i] = g3v - det - gl;
}


void launch_cumulants(int nA, const double* G1, const double* G2, const double* g3, double* L2,
                      double* L3, double* eta, hipStream_t st) {
  int n = 2 * nA;
  if (n == 0) return;
  long long t2 = (long long)n * n * n * n;
  hipLaunchKernelGGL(cumulant2_kernel, dim3((unsigned)((t2 + 255) / 256)), dim3(256), 0, st, n, G1,
                     G2, L2, eta);
  if (g3 && L3) {
    const int n3 = n * n * n;
    hipLaunchKernelGGL(cumulant3_kernel, dim3((unsigned)n3, (unsigned)((n3 + 255) / 256)), dim3(256), 0, st,
                       n, G1, L2, g3, L3);
  }
}

// ---------------------------------------------------------------------------
// Regulariser and source factor (FP64 throughout)
// R_s(D) = (1 - exp(-s D^2)) / D, evaluated as -expm1(-s D^2) / D; R_s(0) = 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double regulariser(double s, double D) {
  if (D == 0.0) return 0.0;
  if (isinf(s)) return 1.0 / D;
  return -expm1(-s * D * D) / D;
}
__device__ __forceinline__ double source_factor(double s, double D) {
  if (isinf(s)) return D == 0.0 ? 1.0 : 0.0;
  return exp(-s * D * D);
}

// element index in 32-bit arithmetic when the block has fewer than 2^31 elements (Idx =
// unsigned), else 64-bit
template <class Idx>
__global__ void first_order_doubles_kernel(AmpDims d, const double* __restrict__ J,
                                           const double* __restrict__ eps, const double* __restrict__ sp,
                                           double* __restrict__ Taa, double* __restrict__ Tab,
                                           double* __restrict__ Yaa, double* __restrict__ Yab,
                                           double* __restrict__ Eaa, double* __restrict__ Eab) {
  const double s = *sp;
  const int nH = d.nC + d.nA, nP = d.nA + d.nV;
  const Idx total = (Idx)nP * nP * nH * nH;
  const Idx idx = (Idx)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const Idx q1 = idx / nH, q2 = q1 / nH, q3 = q2 / nP;
  const int j = (int)(idx - q1 * nH), i = (int)(q1 - q2 * nH), b = (int)(q2 - q3 * nP), a = (int)q3;
  // J(HP|HP)[i][a][j][b] = (ia|jb) = (ai|bj)
  double vab = J[(((long long)i * nP + a) * nH + j) * nP + b];
  double vx = J[(((long long)j * nP + a) * nH + i) * nP + b];  // (aj|bi)
  double vaa = vab - vx;
  bool internal = a < d.nA && b < d.nA && i >= d.nC && j >= d.nC;
  double D = eps[i] + eps[j] - eps[d.nC + a] - eps[d.nC + b];
  double R = regulariser(s, D);
  double tab = internal ? 0.0 : vab * R, taa = internal ? 0.0 : vaa * R;
  Tab[idx] = tab;
  Taa[idx] = taa;
  Yab[idx] = -D * tab;
  Yaa[idx] = -D * taa;
  Eab[idx] = 2.0 * vab - D * tab;
  Eaa[idx] = 2.0 * vaa - D * taa;
}

void launch_first_order_doubles(AmpDims d, const double* J, const double* eps, const double* s,
                                double* T2aa, double* T2ab, double* Y2aa, double* Y2ab,
                                double* E2aa, double* E2ab, hipStream_t st) {
  long long nH = d.nC + d.nA, nP = d.nA + d.nV;
  long long total = nP * nP * nH * nH;
  if (total == 0) return;
  if (total < (1LL << 31))
    hipLaunchKernelGGL(first_order_doubles_kernel<unsigned>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, d, J, eps, s, T2aa, T2ab, Y2aa, Y2ab, E2aa, E2ab);
  else
    hipLaunchKernelGGL(first_order_doubles_kernel<long long>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, d, J, eps, s, T2aa, T2ab, Y2aa, Y2ab, E2aa, E2ab);
}

// coup_a[a,i] = sum_ux (e_x - e_u)(t_aa[a,x,i,u] g_a[x,u] + t_ab[a,x,i,u] g_b[x,u])
// coup_b[a,i] = sum_ux (e_x - e_u)(t_bb[a,x,i,u] g_b[x,u] + t_ab[x,a,u,i] g_a[x,u])
__global__ void singles_kernel(AmpDims d, const double* __restrict__ Taa, const double* __restrict__ Tab,
                               const double* __restrict__ Tbb, const double* __restrict__ ga,
                               const double* __restrict__ gb, const double* __restrict__ eps, const double* __restrict__ sp,
                               const double* __restrict__ fa, const double* __restrict__ fb,
                               const double* __restrict__ za, const double* __restrict__ zb,
                               double* __restrict__ t1a, double* __restrict__ t1b,
                               double* __restrict__ srca, double* __restrict__ srcb) {
  const double s = *sp;
  const int nH = d.nC + d.nA, nP = d.nA + d.nV, nA = d.nA, nC = d.nC;
  // one wave per element, lane l takes the terms l, l + 64, ... (u * nA + x) of the active
  // sum (one term each for nA <= 8), summed by a fixed butterfly
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (idx >= 2 * nP * nH) return;   // the whole wave
  int spin = idx / (nP * nH);
  int e = idx - spin * nP * nH;
  int a = e / nH, i = e % nH;
  double c = 0.0;
  const long long sH = 1, sH2 = nH, sP = (long long)nH * nH, sP2 = (long long)nP * nH * nH;
  for (int l = lane; l < nA * nA; l += 64) {
    const int u = l / nA, x = l - u * nA;
    double D = eps[nC + x] - eps[nC + u];
    // t[a, x, i, u]: a (P), x (P, active at offset 0), i (H), u (H, active at offset nC)
    long long o_axiu = a * sP2 + x * sP + i * sH2 + (nC + u) * sH;
    if (spin == 0) {
      c += D * (Taa[o_axiu] * ga[x * nA + u] + Tab[o_axiu] * gb[x * nA + u]);
    } else {
      long long o_xaui = x * sP2 + a * sP + (nC + u) * sH2 + i * sH;
      c += D * (Tbb[o_axiu] * gb[x * nA + u] + Tab[o_xaui] * ga[x * nA + u]);
    }
  }
  for (int w = 32; w > 0; w >>= 1) c += __shfl_xor(c, w, 64);
  if (lane != 0) return;
  double f = 0.0;
  const double* fp = spin ? fb : fa;
  const double* zp = spin ? zb : za;
  if (fp) f = zp ? fp[e] + 0.5 * zp[e] : fp[e];
  bool internal = a < nA && i >= nC;
  double D1 = eps[i] - eps[nC + a];
  double* t1 = spin ? t1b : t1a;
  double* src = spin ? srcb : srca;
  t1[e] = internal ? 0.0 : (f + c) * regulariser(s, D1);
  if (src) src[e] = internal ? 0.0 : (f + c) * source_factor(s, D1);
}

void launch_singles(AmpDims d, const double* T2aa, const double* T2ab, const double* T2bb,
                    const double* g1a, const double* g1b, const double* eps, const double* s,
                    const double* fa, const double* fb, double* t1a, double* t1b, double* srca,
                    double* srcb, hipStream_t st, const double* za, const double* zb) {
  int nH = d.nC + d.nA, nP = d.nA + d.nV;
  int total = 2 * nP * nH;   // elements, one wave each
  if (total == 0) return;
  hipLaunchKernelGGL(singles_kernel, dim3((total + 3) / 4), dim3(256), 0, st, d, T2aa, T2ab, T2bb,
                     g1a, g1b, eps, s, fa, fb, za, zb, t1a, t1b, srca, srcb);
}

// Spin block blockIdx.y; the element index in 32-bit arithmetic when a block has fewer than
// 2^31 elements (Idx = unsigned), else 64-bit.
template <class Idx>
__global__ void second_order_doubles_kernel(AmpDims d, const double* __restrict__ W,
                                            const double* __restrict__ Z,
                                            const double* __restrict__ eps, const double* __restrict__ sp,
                                            double* __restrict__ U, double* __restrict__ H) {
  const double s = *sp;
  const Idx nH = d.nC + d.nA, nP = d.nA + d.nV;
  const Idx total = nP * nP * nH * nH;
  const Idx idx = (Idx)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const long long o = (long long)blockIdx.y * (long long)total + (long long)idx;
  const Idx q1 = idx / nH, q2 = q1 / nH, q3 = q2 / nP;
  const int j = (int)(idx - q1 * nH), i = (int)(q1 - q2 * nH), b = (int)(q2 - q3 * nP), a = (int)q3;
  const bool internal = a < d.nA && b < d.nA && i >= d.nC && j >= d.nC;
  const double D = eps[i] + eps[j] - eps[d.nC + a] - eps[d.nC + b];
  const double z = Z[o];
  const double v2 = W[o] + 0.5 * z;  // (2 W + Z) / 2
  U[o] = internal ? 0.0 : v2 * regulariser(s, D);
  H[o] = (internal ? v2 : v2 * source_factor(s, D)) - z / 6.0;
}

void launch_second_order_doubles(AmpDims d, const double* W, const double* Z, const double* eps,
                                 const double* s, double* U, double* H, int nblocks, hipStream_t st) {
  long long nH = d.nC + d.nA, nP = d.nA + d.nV;
  long long total = nP * nP * nH * nH;
  if (total == 0 || nblocks <= 0) return;
  const dim3 grid((unsigned)((total + 255) / 256), (unsigned)nblocks);
  if (total < (1LL << 31))
    hipLaunchKernelGGL(second_order_doubles_kernel<unsigned>, grid, dim3(256), 0, st, d, W, Z, eps, s, U, H);
  else
    hipLaunchKernelGGL(second_order_doubles_kernel<long long>, grid, dim3(256), 0, st, d, W, Z, eps, s, U, H);
}


// spin block blockIdx.y
__global__ void second_order_h1_kernel(AmpDims d, const double* __restrict__ W1,
                                       const double* __restrict__ Z1,
                                       const double* __restrict__ src, double* __restrict__ H1) {
  const int nH = d.nC + d.nA, nP = d.nA + d.nV;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nP * nH) return;
  int a = e / nH, i = e % nH;
  const long long o = (long long)blockIdx.y * nP * nH + e;
  bool internal = a < d.nA && i >= d.nC;
  double z = Z1[o];
  double f2 = W1[o] + 0.5 * z;
  H1[o] = (internal ? f2 : src[o]) - z / 6.0;
}

void launch_second_order_h1(AmpDims d, const double* W1, const double* Z1, const double* src,
                            double* H1, int nspins, hipStream_t st) {
  int n = (d.nA + d.nV) * (d.nC + d.nA);
  if (n == 0 || nspins <= 0) return;
  hipLaunchKernelGGL(second_order_h1_kernel, dim3((n + 255) / 256, (unsigned)nspins), dim3(256), 0, st, d, W1,
                     Z1, src, H1);
}

__global__ __launch_bounds__(256) void pair_dot_kernel(AmpDims d, const double* __restrict__ G2,
                                                       const double* __restrict__ Taa,
                                                       const double* __restrict__ Tab,
                                                       const double* __restrict__ Tbb,
                                                       double* __restrict__ P2) {
  __shared__ double red[256];
  const int nH = d.nC + d.nA, nP = d.nA + d.nV;
  const int i = blockIdx.x / d.nC, j = blockIdx.x - i * d.nC;
  const long long n4 = (long long)nP * nP * nH * nH;
  const long long nab = (long long)nP * nP;
  double part = 0.0;
  for (long long e = threadIdx.x; e < 3 * nab; e += 256) {
    const int blk = (int)(e / nab);
    const long long ab = e - blk * nab;
    const long long o = (ab * nH + i) * nH + j;
    const double* T = blk == 0 ? Taa : (blk == 1 ? Tab : Tbb);
    part += G2[blk * n4 + o] * T[o];
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) P2[i * d.nC + j] += red[0];
}

void launch_pair_dot(AmpDims d, const double* G2, const double* Taa, const double* Tab,
                     const double* Tbb, double* P2, hipStream_t st) {
  if (d.nC <= 0 || d.nA + d.nV <= 0) return;
  hipLaunchKernelGGL(pair_dot_kernel, dim3((unsigned)(d.nC * d.nC)), dim3(256), 0, st, d, G2, Taa, Tab,
                     Tbb, P2);
}

__global__ __launch_bounds__(256) void pair_fold_kernel(int nC, const double* __restrict__ P2,
                                                        const double* __restrict__ energies,
                                                        double* __restrict__ out) {
  __shared__ double red[256];
  const int np = nC * (nC + 1) / 2;
  double part = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) {
    int i = 0, rem = k;
    while (rem >= nC - i) {
      rem -= nC - i;
      ++i;
    }
    const int j = i + rem;
    const double v = i == j ? P2[i * nC + i] : P2[i * nC + j] + P2[j * nC + i];
    out[k] = v;
    part += v;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[np] = (energies[1] + energies[2]) - red[0];
}

void launch_pair_fold(int nC, const double* P2, const double* energies, double* out, hipStream_t st) {
  hipLaunchKernelGGL(pair_fold_kernel, dim3(1), dim3(256), 0, st, nC, P2, energies, out);
}

// one workgroup; thread t sums elements t, t + 256, ... and a fixed tree combines them
__device__ __forceinline__ void weighted_sum_kernel_body(int n, const double* __restrict__ vals,
                                                         const double* __restrict__ coef,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += coef[i] * vals[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(256) void weighted_sum_kernel(int n, const double* __restrict__ vals,
                                                           const double* __restrict__ coef,
                                                           double* __restrict__ out) {
  weighted_sum_kernel_body(n, vals, coef, out);
}

void launch_weighted_sum(int n, const double* vals, const double* coef, double* out, hipStream_t st) {
  hipLaunchKernelGGL(weighted_sum_kernel, dim3(1), dim3(256), 0, st, n, vals, coef, out);
}

// workgroup k: out.o[k] = sum_i coef[k n + i] vals[i], the same fixed order as above
__global__ __launch_bounds__(256) void weighted_sums_kernel(int n, const double* __restrict__ vals,
                                                            const double* __restrict__ coef, SumOuts out) {
  weighted_sum_kernel_body(n, vals, coef + (long long)blockIdx.x * n, out.o[blockIdx.x]);
}

void launch_weighted_sums(int n, const double* vals, const double* coef, const SumOuts& out, hipStream_t st) {
  if (out.n <= 0) return;
  hipLaunchKernelGGL(weighted_sums_kernel, dim3((unsigned)out.n), dim3(256), 0, st, n, vals, coef, out);
}

__global__ void fill_kernel(double* __restrict__ p, long long n, double v) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) p[i] = v;
}

void launch_fill(double* p, long long n, double v, hipStream_t st) {
  if (n <= 0) return;
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

// Excitation block of the inter-block Fock matrix: F1[a][i] = f[nC + a][i] for a in P,
// i in H, zero on internal (active-active) elements, which f(1) does not have.
__global__ __launch_bounds__(256) void fock_exc_kernel(AmpDims d, const double* __restrict__ f,
                                                       double* __restrict__ F1) {
  const int nH = d.nC + d.nA, nP = d.nA + d.nV, N = d.nC + d.nA + d.nV;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nP * nH) return;
  const int a = e / nH, i = e - a * nH;
  const bool internal = a < d.nA && i >= d.nC;
  F1[e] = internal ? 0.0 : f[(long long)(d.nC + a) * N + i];
}

void launch_fock_exc(AmpDims d, const double* f, double* F1, hipStream_t st) {
  const int n = (d.nA + d.nV) * (d.nC + d.nA);
  if (n <= 0) return;
  hipLaunchKernelGGL(fock_exc_kernel, dim3((n + 255) / 256), dim3(256), 0, st, d, f, F1);
}

// Y = src - F and E = src + F for nspins one-body blocks of n elements (F shared by the
// spins); Y overwrites src.
__global__ __launch_bounds__(256) void split_source_kernel(long long n, int nspins, double* __restrict__ Y,
                                                           double* __restrict__ E, const double* __restrict__ F) {
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n * nspins; e += 256LL * gridDim.x) {
    const double src = Y[e], f = F[e % n];
    Y[e] = src - f;
    E[e] = src + f;
  }
}

void launch_split_source(long long n, int nspins, double* Y, double* E, const double* F, hipStream_t st) {
  const long long tot = n * nspins;
  if (tot <= 0) return;
  const long long blocks = std::min<long long>((tot + 255) / 256, 16384);
  hipLaunchKernelGGL(split_source_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, nspins, Y, E, F);
}

// dst = src with the elements of core-core hole pairs (i < nC and j < nC) set to zero, over
// nblocks [P][P][H][H] blocks
__global__ __launch_bounds__(256) void mask_core_pairs_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                              long long total, int nH, int nC) {
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < total; e += 256LL * gridDim.x) {
    const long long q = e / nH;
    const int j = (int)(e - q * nH), i = (int)(q % nH);
    dst[e] = (i < nC && j < nC) ? 0.0 : src[e];
  }
}

void launch_mask_core_pairs(AmpDims d, const double* src, double* dst, int nblocks, hipStream_t st) {
  const long long nH = d.nC + d.nA, nP = d.nA + d.nV;
  const long long total = nP * nP * nH * nH * nblocks;
  if (total <= 0) return;
  const long long blocks = std::min<long long>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(mask_core_pairs_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, total, (int)nH, d.nC);
}

// Features of the core pairs i <= j (row-major over the upper triangle), one workgroup per
// pair, from V[a][b] = (ai|bj) and X[a][b] = (bi|aj) over particles a, b (the Coulomb block
// J[i][a][j][b] = (ai|bj)), D = e_i + e_j - e_a - e_b, R = R_s(D), f = exp(-s D^2):
//  0 e_i, 1 e_j, 2 min |D|, 3 mean R, 4 1/(1 + s), 5 log|E2_ij|, 6 log|E2inf_ij|,
//  7 log sum t^2, 8 log (sum V^2 / nP^2), 9 log max|t|, 10 same-spin share of E2_ij,
//  11 log nV, 12 log M, 13 [i == j], 14 log (ii|jj), 15 log (ij|ij)
// with t = V R, E2_ij = c (2 sum V^2 (1 + f) R + sum (V - X)^2 (1 + f) R [i < j]) (c = 1 for
// i < j, 1/2 for i == j), E2inf_ij the same with (1 + f) R -> 1/D.  e2_out[k] = E2_ij.
// Sums in FP64 in a fixed order (a tree over the workgroup).
constexpr int kPairFeatures = 16;
__global__ __launch_bounds__(256) void pair_features_kernel(AmpDims d, const double* __restrict__ J,
                                                            const double* __restrict__ eps, const double* __restrict__ sp,
                                                            const double* __restrict__ B, int M,
                                                            float* __restrict__ feat, double* __restrict__ e2_out) {
  const double s = *sp;
  const int nC = d.nC, nH = d.nC + d.nA, nP = d.nA + d.nV, N = nH + d.nV;
  // pair k -> (i, j), i <= j
  int k = blockIdx.x, i = 0;
  while (k >= nC - i) {
    k -= nC - i;
    ++i;
  }
  const int j = i + k;
  const bool diag = i == j;
  __shared__ double red[8][256];
  double os = 0, ss = 0, osi = 0, ssi = 0, tn = 0, vn = 0, tmax = 0, rs = 0, dmin = 1e300;
  const long long sH = (long long)nP * nH * nP;   // J[i][a][j][b]
  for (long long e = threadIdx.x; e < (long long)nP * nP; e += 256) {
    const int a = (int)(e / nP), b = (int)(e - (long long)a * nP);
    const double V = J[i * sH + (long long)a * nH * nP + (long long)j * nP + b];
    const double X = J[i * sH + (long long)b * nH * nP + (long long)j * nP + a];
    const double D = eps[i] + eps[j] - eps[nC + a] - eps[nC + b];
    const double R = regulariser(s, D), f = source_factor(s, D);
    const double inv = D != 0.0 ? 1.0 / D : 0.0;
    os += V * V * (1.0 + f) * R;
    osi += V * V * inv;
    if (!diag) {
      ss += (V - X) * (V - X) * (1.0 + f) * R;
      ssi += (V - X) * (V - X) * inv;
      tn += 0.5 * (V - X) * (V - X) * R * R;
    }
    tn += V * V * R * R;
    vn += V * V;
    tmax = fmax(tmax, fabs(V * R));
    rs += R;
    dmin = fmin(dmin, fabs(D));
  }
  double v[8] = {os, ss, osi, ssi, tn, vn, rs, tmax};
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = v[q];
  __shared__ double dm[256];
  dm[threadIdx.x] = dmin;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int q = 0; q < 7; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
      red[7][threadIdx.x] = fmax(red[7][threadIdx.x], red[7][threadIdx.x + w]);
      dm[threadIdx.x] = fmin(dm[threadIdx.x], dm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double c = diag ? 0.5 : 1.0;
  const double e2 = c * (2.0 * red[0][0] + red[1][0]);
  const double e2i = c * (2.0 * red[2][0] + red[3][0]);
  double iijj = 0, ijij = 0;
  for (int Q = 0; Q < M; ++Q) {
    const double* BQ = B + (long long)Q * N * N;
    iijj += BQ[(long long)i * N + i] * BQ[(long long)j * N + j];
    ijij += BQ[(long long)i * N + j] * BQ[(long long)i * N + j];
  }
  const double tiny = 1e-300;
  float* o = feat + (long long)blockIdx.x * kPairFeatures;
  o[0] = (float)eps[i];
  o[1] = (float)eps[j];
  o[2] = (float)dm[0];
  o[3] = (float)(red[6][0] / ((double)nP * nP));
  o[4] = (float)(1.0 / (1.0 + s));
  o[5] = (float)log(fabs(e2) + tiny);
  o[6] = (float)log(fabs(e2i) + tiny);
  o[7] = (float)log(red[4][0] + tiny);
  o[8] = (float)log(red[5][0] / ((double)nP * nP) + tiny);
  o[9] = (float)log(red[7][0] + tiny);
  o[10] = (float)(fabs(e2) > 0 ? c * red[1][0] / e2 : 0.0);
  o[11] = (float)log((double)d.nV + 1.0);
  o[12] = (float)log((double)M);
  o[13] = diag ? 1.f : 0.f;
  o[14] = (float)log(fabs(iijj) + tiny);
  o[15] = (float)log(ijij + tiny);
  e2_out[blockIdx.x] = e2;
}

void launch_pair_features(AmpDims d, const double* J, const double* eps, const double* s, const double* B, int M,
                          float* feat, double* e2, hipStream_t st) {
  const int np = d.nC * (d.nC + 1) / 2;
  if (np <= 0) return;
  hipLaunchKernelGGL(pair_features_kernel, dim3(np), dim3(256), 0, st, d, J, eps, s, B, M, feat, e2);
}

__global__ __launch_bounds__(256) void add_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                                  long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) dst[i] += src[i];
}

void launch_add(double* dst, const double* src, long long n, hipStream_t st) {
  if (n <= 0) return;
  const long long blocks = std::min<long long>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
}

}  // namespace dsrg
