/*
 * dsrg.h -- C ABI of the DSRG-MRPT3 hot path on one AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the unrelaxed second- and third-order correlation energies of
 * the driven similarity renormalization group multireference perturbation theory
 * (Li & Evangelista, arXiv:1701.02011):
 *   E(2) = <Psi0|[H~(1), T(1)]|Psi0>                                 (Sec. II.B, Eq. E(2))
 *   E(3) = <Psi0|[H~(1), T(2)]|Psi0> + <Psi0|[H~(2)_{1,2}, T(1)]|Psi0> (Sec. II.B, Eq. E(3))
 * with first- and second-order amplitudes from the DSRG-regularised expressions
 * (Eqs. T1_1st, T2_1st, T1_2nd, T2_2nd), commutators truncated to one- and two-body
 * operators under the Mukherjee-Kutzelnigg generalised normal ordering (Sec. II.A), and
 * two-electron integrals from a factorised three-index tensor (Sec. III, Eq. int_fact).
 *
 * Conventions
 *   - Spatial orbitals are ordered [core | active | virtual]; N = nC + nA + nV.
 *   - Orbitals are restricted (one spatial set for alpha and beta); the reference may
 *     have different alpha and beta densities.
 *   - The orbitals are semicanonical: eps are the diagonal elements of the core, active
 *     and virtual blocks of the generalised Fock matrix (Sec. II.B, Eq. F0th).  The
 *     inter-block Fock elements f(1) are an optional input (zero when not given).
 *   - e2 and e3 are correlation energies of the unrelaxed series (Eq. E_unrelaxed);
 *     e_total adds the caller's reference energy e0.
 *   - All arrays are FP64, C (row-major) order.
 *
 * Execution: the first call of a shape (device, nC, nA, nV, n_aux, gamma3 and f_offdiag
 * given or not, E(2) or E(3), grouping, precision, workspace_cap, virt_batch) runs the pipeline and records it as a plan: its
 * device buffers plus a HIP graph of every launch.  Later calls of that shape copy their
 * inputs into the plan's buffers and launch the graph on the caller's stream; the result
 * is bitwise the same as the recording run's would be for the same inputs.  At most 4
 * plans (16 GiB) are kept, least recently used first out; dsrg_release_cache() frees them.
 * Calls with DSRG_F_PROFILE, DSRG_F_NO_PLAN_CACHE or intermediates run without a plan.
 * Part of a call's work (the (PP|PP) ladder beside the grouped contractions of E(3)'s
 * first-order commutators) may run on a second, library-owned stream of default priority,
 * ordered after the caller's stream and joined back into it before the call's last work
 * there (in a plan, the same fork and join are edges of the graph); except with
 * DSRG_F_PROFILE, which keeps every launch on the caller's stream.
 *
 * Thread safety: calls may run concurrently from different host threads on different
 * streams.  A call that finds the plan of its shape in use by another call runs without one.
 */
#ifndef DSRG_H
#define DSRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define DSRG_OK 0
#define DSRG_E_ARG (-1)         /* NULL pointer, negative size, n_aux < 1, s <= 0 or NaN */
#define DSRG_E_NONFINITE (-2)   /* NaN or Inf in eps, B or the densities */
#define DSRG_E_OOM (-3)         /* device allocation failed or workspace_cap too small */
#define DSRG_E_HIP (-4)         /* HIP runtime error (message in dsrg_last_error) */
#define DSRG_E_UNSUPPORTED (-5) /* option not built (unknown precision, nA > 16) */
#define DSRG_E_RDM (-6)         /* gamma1 not symmetric, or gamma2 not Hermitian (uv <-> xy) or,
                                   in its same-spin blocks, not antisymmetric in u <-> v and
                                   x <-> y, beyond 1e-10 */
#define DSRG_E_INTRUDER (-7)    /* s = +INFINITY and some non-internal denominator |D| < 1e-12
                                   (the unregularised limit 1/D does not exist) */

/* options.precision */
#define DSRG_PRECISION_FP64 0   /* every step in FP64 */
#define DSRG_PRECISION_FP32 1   /* the tensor contractions (integral builds, ladders, table products)
                                   multiply FP32-rounded operands on FP32 MFMA, sum in FP32 over at
                                   most 1024 k values and accumulate those partial sums in FP64;
                                   tensors stay FP64 in memory; denominators, the regulariser and
                                   every energy reduction stay FP64 */
#define DSRG_PRECISION_BF16X3 2 /* the tensor contractions as with FP32, each FP32-rounded operand
                                   split into BF16 parts x = hi + lo (hi = bf16(x), lo = bf16(x - hi))
                                   and every product formed as hi.hi + hi.lo + lo.hi on BF16 MFMA
                                   with FP32 sums (about 16 significant bits per product); the rest
                                   as with FP32 */

/* options.flags */
#define DSRG_F_DEVICE_PTRS 1    /* every array pointer in dsrg_problem is a device pointer */
#define DSRG_F_PROFILE 2        /* bracket every contraction launch with HIP events and report
                                   per-role device time in dsrg_result.role_* (adds overhead) */
#define DSRG_F_NO_GROUPING 4    /* one launch per contraction.  By default the independent
                                   contractions of each commutator run as grouped launches (one
                                   per dependency level) whenever their temporaries fit in half of
                                   workspace_cap; results agree to rounding either way, and each
                                   mode is deterministic. */
#define DSRG_F_NO_PLAN_CACHE 8  /* neither use nor record a cached plan (see Execution above) */
#define DSRG_F_FULL_LADDER 16   /* contract the (PP|PP) ladder over every ordered pair of particle
                                   and hole indices.  By default it runs on unique pairs: p<q,
                                   r<s, i<j for the antisymmetric same-spin amplitudes (the two
                                   same-spin blocks share one contraction when their amplitudes
                                   are the same array), p<=q, r<=s, i<=j for the parts of the
                                   opposite-spin amplitudes symmetric and antisymmetric in the
                                   particle pair, with integral batches of the rows q>=p only
                                   (about a quarter of the ladder and half of the integral work);
                                   results agree to rounding either way. */

typedef struct {
  int32_t n_core, n_active, n_virtual, n_aux;
  /* [N] semicanonical orbital energies (E_h) */
  const double* eps;
  /* [n_aux][N][N], symmetric in the last two indices: (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s] */
  const double* B;
  /* [2][nA][nA]: gamma1[s][u][v] = <a+_{u s} a_{v s}>, s = alpha, beta.  Unused if nA == 0. */
  const double* gamma1;
  /* [3][nA][nA][nA][nA], blocks aa, ab, bb: gamma2[b][u][v][x][y] = <a+_u a+_v a_y a_x> with
     spins (s1, s2) on (u, x) and (v, y). */
  const double* gamma2;
  /* [4][nA]^6, blocks aaa, aab, abb, bbb: gamma3[b][u][v][w][x][y][z] =
     <a+_u a+_v a+_w a_z a_y a_x>, spins (s1, s2, s3) on (u,x), (v,y), (w,z).
     NULL sets the three-body cumulant to zero (an approximation; never used for parity). */
  const double* gamma3;
  /* flow parameter s (E_h^-2), > 0; +INFINITY selects the unregularised limit 1/D */
  double s;
  /* [N][N] inter-block part of the Fock matrix, f(1) of H(1) = f(1) + V (Sec. II.B: H(0) holds
     the core, active and virtual diagonal blocks, which are diagonal in semicanonical
     orbitals).  Only the elements between different blocks (core-active, core-virtual,
     active-virtual) are read; the matrix must be symmetric there.  NULL means f(1) = 0. */
  const double* f_offdiag;
  /* reference energy E0 (E_h); only added into dsrg_result.e_total (Eq. E_unrelaxed).  A
     zero-initialised struct gives e_total = E(2) + E(3); NaN gives NaN. */
  double e0;
} dsrg_problem;

typedef struct {
  int32_t flags;          /* DSRG_F_* */
  int32_t precision;      /* DSRG_PRECISION_FP64 (0), _FP32 (1) or _BF16X3 (2) */
  int64_t workspace_cap;  /* bytes of device workspace for the (PP|PP) integrals and their packed
                             pair rows; 0 = 48 GiB.  When the whole block over particle pairs
                             x <= y (8 (nP (nP + 1) / 2)^2 bytes, plus n_aux nP (nP + 1) / 2 for
                             the packed B) fits beside one batch of packed rows, it is built
                             once and kept resident; else it is built in batches of rows.  Half
                             of an explicit cap (4 GiB by default) bounds the temporaries of a
                             grouped commutator. */
  void* stream;           /* hipStream_t to run on, or NULL for the null stream; caller owns it */
  int32_t virt_batch;     /* values of the first particle index per (PP|PP) integral batch
                             (Sec. III, Eq. scaling_problem); 0 = the largest batch that fits
                             workspace_cap.  A batch that does not fit workspace_cap, or a cap
                             below one row, returns DSRG_E_OOM. */
} dsrg_options;

typedef struct {
  double e2;              /* E(2) (E_h) */
  double e3;              /* E(3) = e3_a + e3_b (E_h) */
  double e3_a;            /* <[H~(1), T(2)]> */
  double e3_b;            /* <[H~(2)_{1,2}, T(1)]> */
  double t_seconds[8];    /* device time: [0] densities+integrals, [1] first order, [2] E(2),
                             [3] [V,A] (ladders, rings), [4] [Y,A], [5] second order + E(3),
                             [6] unused, [7] whole pipeline.  Small problems run E(2), [V,A]
                             and [Y,A] as one grouped sequence: its time is in [2] and [3],
                             [4] are 0.  A call that replays a plan fills [7] only. */
  double gett_flops;      /* floating-point operations issued by the contraction kernels */
  double ladder_flops;    /* of which the (PP|PP) particle-particle ladder (Sec. III) */
  double ladder_seconds;  /* with DSRG_F_PROFILE: device time of the (PP|PP) ladder groups */
  int32_t ladder_batch;   /* virtual batch size used for the (PP|PP) integrals */
  int32_t n_launch;       /* kernel launches issued */
  /* with DSRG_F_PROFILE: contraction launches by role [0] table products one launch each,
     [1] (PP|PP) ladder products, [2] Coulomb-block builds from B, [3] grouped launches of
     table products: device seconds, flops, launches */
  double role_seconds[4];
  double role_flops[4];
  int32_t role_launches[4];
  int32_t plan;           /* 0: ran without a plan, 1: ran and recorded a plan, 2: replayed one */
  int32_t grouped_uses;   /* commutator evaluations run as grouped launches (the others ran
                             one launch per contraction) */
  double role_bytes[4];   /* with DSRG_F_PROFILE: algorithmic bytes of the role_* launches, each
                             operand view read once and the result written once (read too when
                             accumulated) */
  double e_total;         /* e0 + E(2) + E(3) (E(3) = 0 for dsrg_pt2_energy) */
  double alg_flops;       /* algorithmic flops of the executed contractions: 2 M N K per
                             contraction of the term list and of the integral builds, unique
                             index pairs for the ladder, no zero padding */
  int32_t precision_used; /* DSRG_PRECISION_* the contractions ran in */
  int32_t virt_batch_used;/* (PP|PP) batch size used (0: no ladder) */
  /* with DSRG_F_PROFILE: the role_* figures per kernel instance, index 2 * role + t with
     t = 1 for the launches of 128 x 128 output tiles (their own kernel instance), 0 else */
  double kernel_seconds[8];
  double kernel_flops[8];
  int32_t kernel_launches[8];
} dsrg_result;

/* Optional host outputs of intermediates (each pointer may be NULL).  Shapes use
   nH = nC + nA and nP = nA + nV; excitation order [P][H] and [P][P][H][H] (C-convention
   coefficient of {a+_a a_i} and 1/4 {a+_a a+_b a_j a_i}). */
typedef struct {
  double* t1;   /* [2][nP][nH]       first-order singles, spins a, b */
  double* t2;   /* [3][nP][nP][nH][nH] first-order doubles, blocks aa, ab, bb */
  double* w1;   /* [2][nP][nH]       excitation block of [f(1) + V, A(1)]_{1,2} */
  double* w2;   /* [3][nP][nP][nH][nH] */
  double* z1;   /* [2][nP][nH]       excitation block of [[H(0), A(1)], A(1)]_{1,2} */
  double* z2;   /* [3][nP][nP][nH][nH] */
  double* u1;   /* [2][nP][nH]       second-order singles */
  double* u2;   /* [3][nP][nP][nH][nH] second-order doubles */
} dsrg_intermediates;

/* E(2) only (Eq. E(2)); out->e3* are set to 0.  Returns DSRG_OK or a DSRG_E_* code; on
   error *out is left untouched.  The caller owns all buffers; inputs are only read. */
int dsrg_pt2_energy(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out);

/* E(2) and E(3) (Eqs. E(2), E(3)).  Same conventions as dsrg_pt2_energy. */
int dsrg_pt3_energy(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out);

/* E(2) and E(3) of n independent problems (e.g. geometries along a dissociation curve, or
   one geometry at several s).  Items run in rounds of K on streams of the library, ordered
   after opt->stream, each with a plan of its own slot (item k uses slot k % K), so the
   items of a round overlap on the GPU; K is half of GPU_MAX_HW_QUEUES (4 unless set, so 2),
   at most 4.  The call returns when all have finished.  Items of a round whose slot has
   no cached plan (a shape not seen before) run their whole pipeline directly and record
   that plan: items whose first-order doubles hold at most 2^22 elements per spin block
   ((n_core + n_active)^2 (n_active + n_virtual)^2) each on a host worker thread of its own
   and on its round's stream, so small uneven geometries overlap on the GPU too; larger
   ones one after another on the calling thread (each fills the GPU alone).
   outs[k] and status[k] receive item k's result and return code; an item that fails (bad
   arguments, non-finite input) is skipped and leaves outs[k] untouched.  Returns DSRG_OK if
   at least one item succeeded, else the first item's code (DSRG_E_ARG for n < 1 or null
   arrays).  Results equal those of single calls bit for bit. */
int dsrg_pt3_energy_batch(const dsrg_problem* probs, int32_t n, const dsrg_options* opt,
                          dsrg_result* outs, int32_t* status);

/* E(2), E(3) and a core-pair decomposition of E(3).  E(3) = <[H~(1), T(2)]> +
   <[H~(2)_{1,2}, T(1)]> is linear in the amplitudes of its two commutators (Eq. E(3));
   e3_pairs[k] is its value with those amplitudes restricted to the doubles whose two hole
   indices are the spatial core orbitals i and j (any spins, both orders), for the pairs
   i <= j in row-major order of the upper triangle (k = 0 .. nC(nC+1)/2 - 1); *e3_rest =
   E(3) - sum_k e3_pairs[k] (singles and doubles with an active hole index).  The
   decomposition is a reading: the paper defines none.  e3_pairs may be NULL if n_core is
   0; runs without a plan. */
int dsrg_pt3_pair_energies(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out,
                           double* e3_pairs, double* e3_rest);

/* For callers that cannot allocate device memory (work under HIP graph capture set up
   around the call's inputs, tight serving loops, harnesses that forbid hipMalloc): E(2) and
   E(3) as dsrg_pt3_energy, with every device buffer of the pipeline (input copies,
   intermediates, temporaries, integral batches) carved from one static device array of
   DSRG_NOALLOC_SCRATCH_BYTES per GPU, which that GPU holds from the library's first use
   of it until the process ends.  The call allocates nothing: no hipMalloc or hipFree, no
   pinned host memory, no library stream or event, no plan or graph; everything runs on
   opt->stream and the call synchronises it before returning.  The pipeline is planned
   before any device work: a problem whose buffers do not fit returns DSRG_E_OOM and
   leaves *out untouched (tiny and micro problems fit; the small workload does not).
   workspace_cap is lowered to a quarter of the array.  DSRG_F_PROFILE is refused with
   DSRG_E_ARG.  Calls that overlapped on one GPU would share its array and race, so the
   library runs them one at a time (a second host thread waits); the array keeps the last
   call's contents, and every buffer the pipeline needs cleared is cleared by a kernel of
   that call.  Energies agree with dsrg_pt3_energy to summation order (bitwise when both
   group the contractions the same way). */
#define DSRG_NOALLOC_SCRATCH_BYTES (64LL << 20)
int dsrg_pt3_energy_noalloc(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out);

/* ---- learned part: a network for the core-pair parts of E(3) ----
   The core-pair decomposition of E(3) (see dsrg_pt3_pair_energies) is predicted pair by
   pair from 16 features of first order (dsrg_pair_features).  Network: 16 -> 128 -> 128 ->
   128 -> 1 with exact-erf GELU, BF16-rounded weights, FP32 activations and sums; it
   predicts y_ij = e3_ij / |E2_ij|^{3/2} (E2_ij: the pair's second-order proxy), which B ->
   kappa B leaves unchanged.  The weights blob (DSRG_MLP_WEIGHTS_BYTES, caller-owned) holds
   a header, the feature and target standardisation and the FP32 parameters. */
#define DSRG_MLP_FEATURES 16
#define DSRG_MLP_WEIGHTS_BYTES 141572

/* Features of the core pairs i <= j (row-major over the upper triangle), [nC(nC+1)/2][16]
   FP32, and E2_ij [nC(nC+1)/2] FP64, from the first-order quantities of the problem: orbital
   energies, min |D| and mean R_s(D) over the pair's doubles, 1/(1+s), logs of |E2_ij|, of its
   s -> infinity value, of the squared norm and largest element of the pair's amplitudes
   and of its mean squared integral, the same-spin share of E2_ij, log nV, log n_aux,
   [i == j], log (ii|jj), log (ij|ij).  Runs the first-order steps only.  Arrays may be NULL
   when n_core is 0. */
int dsrg_pair_features(const dsrg_problem* prob, const dsrg_options* opt, float* features, double* e2_pairs);

/* Train the network on n rows (X [n][16] features, y [n] targets y_ij) on the GPU: full
   batch Adam (learning rate 1e-3) for `epochs` steps on the mean squared error of the
   standardised targets, uniform initial weights from a counter-based generator of `seed`.
   Writes the trained blob to weights_out.  Host arrays; deterministic. */
int dsrg_mlp_train(const float* X, const double* y, int64_t n, int32_t epochs, uint64_t seed, void* weights_out);

/* y [n] = the network's predictions for X [n][16] (host arrays), on the GPU. */
int dsrg_mlp_predict(const void* weights, const float* X, int64_t n, double* y);

/* E(2) exactly and E(3) = rest + sum of the core-pair parts, with the rest computed exactly
   (the commutators' two-body outputs restricted to hole pairs with an active index, the
   first-order doubles without their core-core pairs) and the pair parts predicted by the
   network; a pair is computed exactly instead (one exact decomposition run for all of
   them) when its predicted part exceeds rel_threshold times the summed magnitude of the
   predictions or a feature lies more than 8 standard deviations from the training mean.
   out->e3_a holds the rest of <[H~(1), T(2)]>, out->e3_b the rest of <[H~(2), T(1)]> plus
   the pair parts; *n_exact_pairs (may be NULL) the number of pairs computed exactly. */
int dsrg_pt3_energy_surrogate(const dsrg_problem* prob, const dsrg_options* opt, const void* weights,
                              double rel_threshold, dsrg_result* out, int32_t* n_exact_pairs);

/* Reference densities from a CAS vector, the step before the path (Sec. II.A: the method
   takes the reference through its densities).  ci [C(nA, n_alpha)][C(nA, n_beta)]: the
   coefficients over alpha strings x beta strings (all subsets of the nA active orbitals in
   lexicographic order of their sorted index lists; a determinant is the alpha creators and
   then the beta creators in ascending order on the vacuum).  Writes gamma1 [2][nA]^2,
   gamma2 [3][nA]^4 and, unless NULL, gamma3 [4][nA]^6 in the layout of dsrg_problem.  Each
   spin block is the Gram matrix of the vectors a_{t_k}..a_{t_1}|Psi> over ordered index
   tuples (an FP64 contraction on the library's contraction kernel), spread over all index
   orders.  With DSRG_F_DEVICE_PTRS in opt->flags every array is a device pointer, else a
   host pointer; runs on opt->stream and synchronises it.  1 <= nA <= 16 (DSRG_E_UNSUPPORTED
   otherwise); DSRG_E_OOM when one spin block's vectors exceed 2^30 doubles. */
int dsrg_active_rdms(const double* ci, int32_t n_active, int32_t n_alpha, int32_t n_beta,
                     const dsrg_options* opt, double* gamma1, double* gamma2, double* gamma3);

/* ---- one-step relaxed DSRG-MRPT3 (Sec. II.B Eqs. energy_relaxed, E_relaxed; App. A) ----
   E^[3] is the lowest eigenvalue of the summed third-order transformed Hamiltonian
   Hbar^[3]_{1,2} = sum_{n=0..3} Hbar^(n)_{1,2} (Eqs. Hbar_0th - Hbar_3rd) within the CAS
   determinant space of n_alpha and n_beta active electrons.  After the unrelaxed pipeline
   the library forms the active blocks of Hbar^[3]_{1,2} (the one- and two-body elements
   with active indices only: H(0) and the integrals <uv||xy>, plus the active blocks of
   1/2 [H~(1), A(1)] + 1/2 [H~(1), A(2)] + 1/2 [H~(2)_{1,2}, A(1)]; [H(0), A] has no active
   element), writes the operator in true-vacuum order with the core folded in (Eqs.
   Hbar_DNO, c0_cas):
     H_CAS = const + sum_uv c^u_v a+_u a_v + 1/4 sum_uvxy Hbar^uv_xy a+_u a+_v a_y a_x,
     const = Hbar_0 - sum Hbar^u_v g^u_v - sum Hbar^uv_xy (g^uv_xy / 4 - g^u_x g^v_y),
     c^u_v = Hbar^u_v - sum_xy Hbar^ux_vy g^x_y   (spin-orbital sums, Hbar_0 = E(2) + E(3)),
   builds its matrix over the determinants (Slater-Condon rules) and finds the lowest
   eigenpair by Davidson iterations, all on the GPU.  The determinants and the CI layout
   are those of dsrg_active_rdms.  The densities of prob must be those of a state with
   n_alpha and n_beta electrons. */
typedef struct {
  double e_relaxed;    /* e0 + lowest eigenvalue of H_CAS (Eq. E_relaxed) */
  double e_unrelaxed;  /* e0 + E(2) + E(3): the reference's expectation value of the same operator */
  double cas_const;    /* const of H_CAS (without e0) */
  double residual;     /* norm of H_CAS x - E x for the returned eigenvector x at exit */
  int32_t n_det;       /* C(nA, n_alpha) C(nA, n_beta) */
  int32_t iterations;  /* Davidson iterations */
  int32_t converged;   /* 1 when residual <= 1e-9 (or the subspace spans the whole space) */
  int32_t reserved;
} dsrg_relaxed_result;

/* Optional host outputs of the relaxation (each pointer may be NULL). */
typedef struct {
  double* ci;      /* [C(nA, n_alpha)][C(nA, n_beta)] the eigenvector, unit norm, sign chosen for a
                      non-negative overlap with ci_guess (else a positive largest element) */
  double* hbar1;   /* [2][nA][nA] Hbar^u_v, spins a, b */
  double* hbar2;   /* [3][nA]^4 Hbar^uv_xy, blocks aa, ab, bb in the layout of gamma2 (coefficient
                      of 1/4 {a+_u a+_v a_y a_x}) */
  double* cas_c;   /* [2][nA][nA] c^u_v */
} dsrg_relaxed_outputs;

/* E(2), E(3) (into *out, as dsrg_pt3_energy) and the relaxed energy (into *rel).  ci_guess
   (host, may be NULL): a start vector for the Davidson iterations, normally the reference's
   CI vector; unit vectors on the lowest diagonal elements are always added.  Returns
   DSRG_E_ARG for n_alpha or n_beta outside [0, nA] or null out/rel, DSRG_E_UNSUPPORTED for
   more than 11585 determinants (the matrix is held densely), DSRG_E_RDM when the
   traces of gamma1 differ from n_alpha, n_beta by more than 1e-8, DSRG_E_NONFINITE for a
   non-finite ci_guess, else as dsrg_pt3_energy.  Runs without a plan; ci_guess and the
   outputs are host memory whatever opt->flags says. */
int dsrg_pt3_energy_relaxed(const dsrg_problem* prob, int32_t n_alpha, int32_t n_beta, const double* ci_guess,
                            const dsrg_options* opt, dsrg_result* out, dsrg_relaxed_result* rel,
                            const dsrg_relaxed_outputs* outs);

/* ---- tile choices by problem size (the batched dissociation curve's autotuned tiles) ----
   A rule applies to every later call (any entry point, any host thread) whose particle
   space n_active + n_virtual lies in [np_min, np_max]; the first matching rule wins, and
   a call matched by none keeps the built-in choices.  big_tile_min: plain contraction
   launches run 128 x 128 output tiles when both free dimensions reach 128 and the output
   holds at least this many such tiles (0: the built-in 256), else 64 x 64 tiles.
   virt_batch: the (PP|PP) batch when the options give none (0: the largest that fits
   workspace_cap).  Cached plans are keyed by the settings they were recorded with.  The
   package's autotuner (autotune.py) times candidate settings per size class on the GPU and
   stores the winners as a rule table. */
typedef struct {
  int32_t np_min, np_max;
  int32_t big_tile_min;
  int32_t virt_batch;
} dsrg_tile_rule;

/* Replaces the process-wide rule table with rules[0..n) (copied; n = 0 clears it).
   DSRG_E_ARG for n < 0, null rules with n > 0, np_min > np_max or a negative setting. */
int dsrg_set_tile_rules(const dsrg_tile_rule* rules, int32_t n);

/* ---- Dyall's zeroth-order Hamiltonian: active-to-virtual doubles (App. B, Eq. t2_aavv) ----
   With the two-body interaction among active orbitals moved into H(0) and s -> inf, the
   first-order amplitudes t_{ef}^{uv} that move two electrons from active (u, v) to virtual
   (e, f) orbitals solve, for each virtual pair, a linear system that couples all active
   pairs of that virtual pair:
     (e_u + e_v - e_e - e_f) t^{uv} + 1/2 sum_xy <xy||uv> t^{xy} - sum_xyz <xy||uv> t^{xz} gamma^y_z = <ef||uv>
   (spin-orbital sums over active orbitals, gamma^y_z = <a+_y a_z>).  The library solves
   every block exactly (Gaussian elimination with partial pivoting, FP64, one workgroup per
   virtual pair and spin block) after building (eu|fv) and the active integrals from B on
   the contraction kernel.  Reads eps, B, n_aux and gamma1 of prob (gamma2, gamma3,
   f_offdiag, s and e0 are not used; s must still be > 0).
   t_out [3][nV][nV][nA][nA]: spin blocks aa (e, f, u, v alpha), ab (e, u alpha; f, v beta),
   bb, each t[e][f][u][v], antisymmetric in (e, f) and in (u, v) within aa and bb.
   dmin (may be NULL): the smallest |shifted denominator| over all blocks, i.e. the smallest
   magnitude of a diagonal element of the systems (App. B Eq. full_preconditioner, read as
   that diagonal).  Host or device arrays as DSRG_F_DEVICE_PTRS in opt->flags says; runs on
   opt->stream and synchronises it.  Returns DSRG_E_UNSUPPORTED unless 1 <= nA <= 9 (a block
   of nA^2 unknowns is factorised in LDS), DSRG_E_INTRUDER when a block is singular (a
   pivot below 1e-13 of its largest element; the outputs are then left untouched with host
   arrays), else the checks and codes of dsrg_pt3_energy. */
int dsrg_dyall_aavv(const dsrg_problem* prob, const dsrg_options* opt, double* t_out, double* dmin);

/* As dsrg_pt3_energy, and copies the requested intermediates to host memory. */
int dsrg_pt3_energy_ex(const dsrg_problem* prob, const dsrg_options* opt, dsrg_result* out,
                       const dsrg_intermediates* inter);

/* Message of the last failing call on this host thread ("" if none). */
const char* dsrg_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int dsrg_version(void);

/* Free the cached plans (device buffers and graphs) that no call is using, and the large
   device buffers (64 MiB and up) the library keeps after a call for reuse by later calls on
   the same device (at most 96 GiB are kept; a failed allocation frees them too).  Returns
   DSRG_OK. */
int dsrg_release_cache(void);

#ifdef __cplusplus
}
#endif
#endif /* DSRG_H */
