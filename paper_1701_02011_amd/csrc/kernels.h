// Device kernels of the DSRG-MRPT3 hot path (gfx950).  Internal interface between the
// executor (dsrg.hip) and the kernels (kernels.hip); not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dsrg {

constexpr int kMaxComp = 6;   // index components per group (M, N or K)
constexpr int kGettBK = 16;   // k step of the contraction kernel (split-K chunks are multiples)
constexpr int kGettBigBK = 32;   // k step of the FP32 / BF16 x3 plain launches with 128 x 128 tiles

// A strided tensor contraction C[m][n] (+)= alpha * sum_k A[m][k] B[k][n], where m, n and
// k are multi-indices (row-major composition of up to kMaxComp components) and every
// operand addresses its elements through its own per-component strides.
//
// The kernel walks k in steps of kGettBK consecutive values of the last k component (the
// "inner" one, zero-padded to a multiple of kGettBK), so inside a step both operands are
// affine in k; the other ("outer") k components advance between steps.  gett_prepare
// merges k components that are contiguous in both operands, picks the inner component and
// the load order; it must run before a launch.
struct GettDesc {
  int M = 1, N = 1, K = 1;
  int nm = 0, nn = 0, nk = 0;
  int md[kMaxComp] = {}, nd[kMaxComp] = {}, kd[kMaxComp] = {};
  long long am[kMaxComp] = {}, ak[kMaxComp] = {};
  long long bk[kMaxComp] = {}, bn[kMaxComp] = {};
  long long cm[kMaxComp] = {}, cn[kMaxComp] = {};
  double alpha = 1.0;
  int beta = 0;        // 0: C = alpha AB, 1: C += alpha AB
  int a_kfast = 1;     // A tile loads walk k fastest (else m fastest)
  int b_kfast = 0;     // B tile loads walk k fastest (else n fastest)
  int ksteps = 1;      // k steps per value of the outer k components
  long long steps = 1;   // total k steps: K / kd[nk - 1] * ksteps (K / (kd[nk-1] kd[nk-2]) * ksteps with kpack)
  // kpack > 1: a step covers kpack consecutive values of component nk - 2 times the whole
  // inner component (kpack * kd[nk - 1] <= kGettBK), for inner components of at most
  // kGettBK / 2 values; ksteps is then the steps per sweep of component nk - 2
  int kpack = 1;
  // tri > 0: output tiles whose last column block (column / tri) lies before their first
  // row block (row / tri) are skipped (left unwritten): blocks of a matrix needed only on and
  // above its block diagonal.  Plain launches only.
  int tri = 0;
  long long kchunk = 1;  // k steps per split (split-K), set by the launcher
  double* part = nullptr;  // split-K partial tiles [split][M][N], set by the launcher
  // tail launches of 128 x 128 tiles (set by the launcher, zero otherwise): the launch covers
  // logical tiles [t0, t0 + nl) of a gx x gy tile grid, and its partial tiles are stored
  // [split][pM][pN] over the box of rows pm0 .. pm0 + pM - 1, columns pn0 .. pn0 + pN - 1
  int gx = 0, gy = 0, t0 = 0, nl = 0;
  int pm0 = 0, pn0 = 0, pM = 0, pN = 0;
  // fewest k steps for 128 x 128 tiles (set by the caller; FP32 and BF16 x3 products walk
  // 32 k values per step there, so short k ranges run faster on 64 x 64 tiles)
  long long big_min_steps = 0;
  // division by md[c] (nd[c]) as a multiply and shift: q = (idx * mmag[c]) >> msh[c] for
  // 0 <= idx < 2^31 (set by gett_magic)
  unsigned mmag[kMaxComp] = {}, nmag[kMaxComp] = {};
  int msh[kMaxComp] = {}, nsh[kMaxComp] = {};
};
// merges and orders components, chooses the inner k component, and sets the magic numbers
void gett_prepare(GettDesc& g);
// fraction of the M x N outputs a plain launch computes (1 unless tri skips tiles)
double gett_tile_fraction(const GettDesc& g);
// whether a plain launch of g runs 128 x 128 tiles (else 64 x 64)
bool gett_big_tiles(const GettDesc& g);
// Tile choice of plain launches on the calling host thread: 128 x 128 tiles when both free
// dimensions reach 128 and the output holds at least big_tile_min such tiles (default 256).
void set_big_tile_min(int n);
int big_tile_min();
// back to plain k steps (for tiles without packed steps)
void gett_unpack_k(GettDesc& g);
// fraction of the k values of all steps that are real (not zero padding)
inline double gett_k_fill(const GettDesc& g) { return (double)g.K / ((double)g.steps * kGettBK); }
// the magic numbers of md and nd alone (after any later change of them)
void gett_magic(GettDesc& g);

// sum_k A[k] B[k] over a strided multi-index k (deterministic two-pass reduction).
// Divisions of a multi-index decode as multiply and shift (see gett_magic), valid for
// indices below 2^31; set on the host (div_magic) before a launch.
struct DivMagic {
  unsigned mag[2 * kMaxComp] = {};
  int sh[2 * kMaxComp] = {};
};
void div_magic(const int* d, int n, DivMagic& m);

struct DotDesc {
  long long K = 0;
  int nk = 0;
  int kd[2 * kMaxComp] = {};
  long long as[2 * kMaxComp] = {}, bs[2 * kMaxComp] = {};
  DivMagic dm;   // of kd (set by the launchers, or by the caller for grouped dots)
};

// out[o] += coef * src[s] over a strided multi-index (rank <= 6).
struct ScatterDesc {
  long long n = 0;
  int rank = 0;
  int d[kMaxComp] = {};
  long long ss[kMaxComp] = {}, so[kMaxComp] = {};
  double coef = 1.0;
  DivMagic dm;   // of d (set by launch_scatter)
};

// Launch roles (same kernel, distinct symbols): contraction-table products, the (PP|PP)
// particle-particle ladder products, and Coulomb-block builds from the DF tensor.  Role 3
// counts the grouped launches of table products (gett_group_kernel) in profiles.
constexpr int kRoleGeneric = 0, kRoleLadder = 1, kRoleIntegrals = 2, kRoleGrouped = 3;
constexpr int kRoles = 4;
// g must have been through gett_prepare.  ws (ws_elems doubles) enables split-K for
// launches with few output tiles and a long k range: partial tiles go to ws and a
// fixed-order reduction writes C (deterministic).
// prec (DSRG_PRECISION_*): 0 FP64 throughout; 1 FP32 products (operands rounded to FP32 in
// LDS, FP32 MFMA); 2 split-BF16 x3 products (operands rounded to FP32 in LDS, split into
// BF16 hi and lo parts, three BF16 MFMAs per block).  With 1 and 2 the FP32 sums are added
// into the FP64 output (or partial tile) every 1024 k values, and 128 x 128 tiles walk
// kGettBigBK k values per step.
void launch_gett(const GettDesc& g, const double* A, const double* B, double* C, hipStream_t st,
                 int role, double* ws, long long ws_elems, int prec = 0);
int gett_splits(const GettDesc& g, long long ws_elems);
// workspace (doubles) for the k-split tail of a 128 x 128 launch without split-K (0 when
// the launch has none): launch_gett splits the k range of the tiles past the last whole
// round of resident workgroups when ws holds this many doubles
long long gett_tail_ws(const GettDesc& g);
// ---- grouped execution: independent contractions of one dependency level per launch ----
// Item i owns workgroup tiles [tile0, tile0 + tiles_m * tiles_n * splits) of a grouped launch,
// each an output tile of shape kGroupTiles[shape] and one chunk of k steps (g.kchunk).
// With splits > 1 the partial tiles go to g.part ([splits][M][N]) and launch_group_reduce
// writes C.
// Shapes 0-2 run in gett_group_kernel, shape 3 (128 x 128, for large items) in a launch of
// its own (launch_gett_group with big = true), since its register count halves occupancy.
constexpr int kGroupShapes = 4, kGroupBigShape = 3;
constexpr int kGroupTiles[kGroupShapes][2] = {{64, 64}, {16, 128}, {128, 16}, {128, 128}};
// Shape 4 (in gett_group_kernel): items with K <= kGettBK and N <= kGroupRowN (the host
// swaps the operands of an item whose short free dimension is M) run one output row per
// thread, kGroupRows rows per workgroup (tiles_n = 1, no split), without LDS tiles or MFMA.
constexpr int kGroupRowShape = 4, kGroupRows = 256, kGroupRowN = 64;
struct GroupItem {
  GettDesc g;
  const double* A = nullptr;
  const double* B = nullptr;
  double* C = nullptr;
  int shape = 0;
  int tiles_m = 0, tiles_n = 0, splits = 1;
  int tile0 = 0;          // first workgroup of this item
};
// tile_item[b] (b < tiles): index of the item that owns workgroup tile b of the launch.
// (coulomb: the same launch under the symbol coulomb_group_kernel, small tiles only)
void launch_gett_group(const GroupItem* items, const int* tile_item, int n, int tiles, bool big,
                       int prec, hipStream_t st, bool coulomb = false);
// Block b of the split-K reduction sums the partial tiles of elements [e0, e0 + 256) of
// item `item` (an index into the launch's items).
struct ReduceBlock {
  int item, e0;
};
void launch_group_reduce(const GroupItem* items, const ReduceBlock* blocks, int nblocks, hipStream_t st);

// Grouped dot products: workgroups [blk0, blk0 + nblk) of the launch sum item i; one
// partial per workgroup.
struct DotItem {
  DotDesc d;
  const double* A = nullptr;
  const double* B = nullptr;
  int blk0 = 0, nblk = 1;
};
void launch_dot_group(const DotItem* items, int n, int blocks, double* partial, hipStream_t st);

// out[x] += sum over the entries of x's class of coef * src[base + sum_k x_k ss[k]], where
// x is a row-major multi-index over dim[0..rank) and the class has bit k set when
// x_k >= split[k].  Entries of class c are [cls[c], cls[c + 1]).
struct GatherEntry {
  const double* src = nullptr;
  long long base = 0;
  long long ss[4] = {};
  double coef = 0;
};
struct GatherDesc {
  int rank = 0;
  int dim[4] = {1, 1, 1, 1};
  int split[4] = {};
  int cls[17] = {};
  int blk[17] = {};   // workgroups of each class (prefix), set by gather_prepare
  const GatherEntry* ent = nullptr;   // this output's entries (classes in order)
  double* out = nullptr;              // contiguous output
  int tpe = 1;                        // lanes per element, set by gather_prepare
  int blk0 = 0;                       // first workgroup of this output in a multi-output launch
};
// lanes per element and class workgroups of one output; returns its workgroup count
long long gather_prepare(GatherDesc& g);
// several outputs (prepared, blk0 their workgroup prefix, the array in device memory) in
// one launch of `blocks` workgroups
// k32: every output has fewer than 2^31 elements and every source offset is below 2^31
void launch_gather_multi(const GatherDesc* descs, int n, long long blocks, hipStream_t st, bool k32 = false);

// partial: scratch of at least dot_partials() doubles; writes the sum into out[0]
int dot_partials();
void launch_dot(const DotDesc& d, const double* A, const double* B, double* partial, double* out,
                hipStream_t st);
void launch_scatter(const ScatterDesc& d, const double* src, double* out, hipStream_t st);

// dst[e] = src[sum_c idx_c(e) ss[c]] with e row-major over d[0..rank) (a packed copy of a
// strided view, rank <= 2 kMaxComp).
struct PackDesc {
  long long n = 0;
  int rank = 0;
  int d[2 * kMaxComp] = {};
  long long ss[2 * kMaxComp] = {};
  DivMagic dm;   // of d (set by launch_pack)
};
void launch_pack(const PackDesc& d, const double* src, double* dst, hipStream_t st);

// ---- (PP|PP) ladder on unique index pairs ----
// A batch of Coulomb integrals holds jb[p - b0][x][q - qoff][y] = (p x|q y) for p in the
// batch, q in [qoff, qoff + nq) and x, y over the particle space.  A pair table entry is a
// pair (a, b) of indices and m, the position of (a, b) among the strict pairs a < b of the
// same table order (-1 when a == b).
struct LadderPair {
  int a, b, m;
};
// Vp[row][k] = (p x|q y) - (p y|q x)              (sym = 0: strict pairs x < y)
// Vp[row][k] = ((p x|q y) + (p y|q x)) w_xy      (sym = 1: pairs x <= y, w = 1/2 on x == y)
// with (p, q) = rowtab[row] and k the position of (x, y) in x-major order of the pairs; every
// q of the rows lies in [qoff, qoff + nq).  With sym = 1 and Va given, the same pass also
// writes the sym = 0 row of every strict pair (m >= 0) into Va[m - m0] (one read of the
// integrals for both parts).
void launch_ladder_pack_v(const double* jb, int nP, int b0, int qoff, int nq, const LadderPair* rowtab,
                          int rows, int sym, double* Vp, hipStream_t st, double* Va = nullptr,
                          long long m0 = 0);
// As launch_ladder_pack_v, reading the integrals from the resident packed block
// K[pair(p, x)][pair(q, y)] = (p x|q y) (pairs a <= b of the nP particle orbitals, a-major;
// K is npk x npk with npk = nP (nP + 1) / 2, both triangles stored).
void launch_ladder_pack_vk(const double* K, int nP, const LadderPair* rowtab, int rows, int sym, double* Vp,
                           hipStream_t st, double* Va = nullptr, long long m0 = 0);
// Bp[Q][pair(a, b)] = B[Q][off + a][off + b] for a <= b < nP (B is [M][N][N])
void launch_pack_pairs(const double* B, int N, int off, int nP, int M, double* Bp, hipStream_t st);
// Fill K[i][j] = K[j][i] (n x n, row-major) where i / blk > j / blk: the blocks a contraction
// with tri = blk skips (blk a multiple of 32)
void launch_mirror_lower(double* K, long long n, int blk, hipStream_t st);
// Tp[n][k] from T [P][P][H][H], (x, y) = ktab[k], (I, J) = ntab[n]:
// mode 0: T[x][y][I][J];  mode 1: (T[x][y][I][J] + T[y][x][I][J]) / 2;
// mode 2: (T[x][y][I][J] - T[y][x][I][J]) / 2
void launch_ladder_pack_t(const double* T, int nP, int nH, const LadderPair* ktab, int kp,
                          const LadderPair* ntab, int np, int mode, double* Tp, hipStream_t st);
// Antisymmetric fill, X = Xp[row * ldx + n] over strict pairs (p, q) = rowtab[row],
// (I, J) = ntab[n], n < np:
// O[p][q][I][J] += c X, O[q][p][I][J] -= c X, O[p][q][J][I] -= c X, O[q][p][J][I] += c X.
// O is [P][P][H][H]; the four elements of distinct (row, n) are distinct.
void launch_ladder_unpack_anti(const double* Xp, int rows, int np, int ldx, const LadderPair* rowtab,
                               const LadderPair* ntab, int nP, int nH, double c, double* O,
                               hipStream_t st);
// Fill from a symmetric part S = Xs[row][n] over pairs p <= q, I <= J (tables rowtab, ntab)
// and an antisymmetric part A = Xa[rowtab[row].m - m0][ntab[n].m] (0 on a diagonal):
// O[p][q][I][J] += c (S + A), O[p][q][J][I] += c (S - A), O[q][p][I][J] += c (S - A),
// O[q][p][J][I] += c (S + A), each image once when p == q or I == J.  npa: row length of Xa.
void launch_ladder_unpack_sym(const double* Xs, const double* Xa, int rows, int np, int npa, int m0,
                              const LadderPair* rowtab, const LadderPair* ntab, int nP, int nH, double c,
                              double* O, hipStream_t st);

// Spin-orbital active densities [2nA]^k from the spin-block inputs, and cumulants.  The
// three-body density enters the cumulant as its spin blocks g3 (expanded on the fly).
void launch_expand_rdm(int nA, int rank, const double* blocks, double* so, hipStream_t st);
// gamma1 (blocks g1 -> G1) and gamma2 (g2 -> G2) in one launch
void launch_expand_rdm12(int nA, const double* g1, double* G1, const double* g2, double* G2, hipStream_t st);
void launch_cumulants(int nA, const double* G1, const double* G2, const double* g3, double* L2,
                      double* L3, double* eta, hipStream_t st);

// The flow parameter s is read from device memory (s points at one double), so a captured
// launch sequence serves every s.
// First-order doubles from the Coulomb block J(HP|HP)[i][a][j][b] = (ai|bj):
// t = v R_s(D), Y = -D t, E = 2 v + Y (E = 2 v on internal elements), blocks aa (=bb) and ab.
struct AmpDims {
  int nC, nA, nV;
};
void launch_first_order_doubles(AmpDims d, const double* Jhphp, const double* eps, const double* s,
                                double* T2aa, double* T2ab, double* Y2aa, double* Y2ab,
                                double* E2aa, double* E2ab, hipStream_t st);
// Singles: coup_s[a,i] = sum_{ux} (e_x - e_u) (t_ss[a,x,i,u] g_s[x,u] + t_{s s'}..[..] g_s'[x,u]);
// t1 = (f + coup) R_s(D), and the non-diagonal one-body source (f + coup) exp(-s D^2).
// f may be null (zero); with za, zb given, f = fa + za / 2 (fb + zb / 2), the second-order
// one-body source (2 W1 + Z1) / 2.  For a null g1 (nA = 0) coup = 0.
void launch_singles(AmpDims d, const double* T2aa, const double* T2ab, const double* T2bb,
                    const double* g1a, const double* g1b, const double* eps, const double* s,
                    const double* fa, const double* fb, double* t1a, double* t1b, double* srca,
                    double* srcb, hipStream_t st, const double* za = nullptr, const double* zb = nullptr);
// Second-order doubles and the H~(2) two-body excitation block:
// O = 2 W + Z; u = (O/2) R_s(D) (0 on internal), H = (O/2) exp(-s D^2) - Z/6 (O/2 - Z/6 internal).
// nblocks spin blocks at a stride of one [P][P][H][H] block, in one launch.
void launch_second_order_doubles(AmpDims d, const double* W, const double* Z, const double* eps,
                                 const double* s, double* U, double* H, int nblocks, hipStream_t st);
// One-body counterpart: f2 = (2 W1 + Z1)/2; H1 = src - Z1/6 (f2 - Z1/6 on internal elements),
// where src = (f2 + coup2) exp(-s D^2) comes from launch_singles.
// nspins blocks at a stride of one [P][H] block, in one launch.
void launch_second_order_h1(AmpDims d, const double* W1, const double* Z1, const double* src,
                            double* H1, int nspins, hipStream_t st);
// P2[i][j] += sum over the blocks aa, ab, bb and a, b in P of G2[blk][a][b][i][j] T[blk][a][b][i][j]
// for core i, j (G2 and T are [P][P][H][H] per block; P2 is [nC][nC]); fixed-order sums.
void launch_pair_dot(AmpDims d, const double* G2, const double* Taa, const double* Tab,
                     const double* Tbb, double* P2, hipStream_t st);
// Core pairs i <= j (row-major over the upper triangle): out[k] = P2[i][j] + P2[j][i]
// (P2[i][i] on the diagonal); out[npairs] = energies[1] + energies[2] - sum_k out[k] in
// a fixed order.
void launch_pair_fold(int nC, const double* P2, const double* energies, double* out, hipStream_t st);
// out = sum_i coef[i] * vals[i] (fixed order)
void launch_weighted_sum(int n, const double* vals, const double* coef, double* out, hipStream_t st);
// out.o[k] = sum_i coef[k][i] vals[i] for k < out.n (<= 8), one launch
struct SumOuts {
  double* o[8] = {};
  int n = 0;
};
void launch_weighted_sums(int n, const double* vals, const double* coef, const SumOuts& out, hipStream_t st);
void launch_fill(double* p, long long n, double v, hipStream_t st);
// F1[a][i] = f[nC + a][i] over a in P, i in H (f is [N][N]); 0 on active-active elements
void launch_fock_exc(AmpDims d, const double* f, double* F1, hipStream_t st);
// Y = src - F, E = src + F over nspins blocks of n elements (Y holds src on entry; F is one
// block shared by the spins)
void launch_split_source(long long n, int nspins, double* Y, double* E, const double* F, hipStream_t st);
// dst = src with the core-core hole pairs (i, j < nC) zeroed, nblocks [P][P][H][H] blocks
void launch_mask_core_pairs(AmpDims d, const double* src, double* dst, int nblocks, hipStream_t st);
// Features of the core pairs i <= j for the pair-energy network (16 per pair, see the
// kernel) from the Coulomb block J(HP|HP)[i][a][j][b] = (ai|bj), eps, s and B; e2[k]: the
// pair's second-order proxy E2_ij
void launch_pair_features(AmpDims d, const double* J, const double* eps, const double* s, const double* B, int M,
                          float* feat, double* e2, hipStream_t st);
// dst[i] += src[i]
void launch_add(double* dst, const double* src, long long n, hipStream_t st);
// O[p][q][i][j] += X[p][q][i][j] - X[q][p][i][j] - X[p][q][j][i] + X[q][p][j][i]
// (both [P][P][H][H], dense, distinct arrays)
void launch_antisym_add(const double* X, double* O, int nP, int nH, hipStream_t st);
// the same for up to kAntisymList pairs (X[k], O[k]) of one shape in one launch (the O
// arrays distinct)
constexpr int kAntisymList = 8;
struct AntisymList {
  const double* X[kAntisymList] = {};
  double* O[kAntisymList] = {};
  int n = 0;
};
void launch_antisym_add_list(const AntisymList& l, int nP, int nH, hipStream_t st);

}  // namespace dsrg
