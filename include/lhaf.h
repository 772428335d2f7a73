/*
 * lhaf.h -- C ABI of the MI355X (gfx950) loop-hafnian library.
 *
 * Computes complex loop hafnians lhaf(A, gamma) of symmetric matrices, their
 * repeated-row ("collision") form and their gradients, following
 * arXiv:2108.01622 (Quesada/Bulmer et al., "The boundary for quantum advantage
 * in Gaussian boson sampling"), App. B:
 *   - lhaf(A) = sum over single-pair matchings of products of A_ij over pairs
 *     and gamma_i over singles (App. B, definition);
 *   - evaluated as a sum over terms of one fixed perfect matching: the
 *     eigenvalue-trace inclusion/exclusion sum (App. B.1, Eqs. ET_loop,
 *     ET_poly) or the finite-difference sieve (App. B.4, Eq. fdsieve), with
 *     repeated pairs (App. B.2) chosen by the greedy matching of App. B.3;
 *   - each term is the lambda^n coefficient of exp(sum_k g_k lambda^k),
 *     g_k = Tr(W^k)/(2k) + u^T W^{k-1} v / 2, W = C X_d (App. B.1/B.2).
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im) doubles: lh_c128 has the layout
 *     of torch.complex128 / hipDoubleComplex.
 *   - Matrices are row-major with leading dimension lda (elements).  The
 *     library reads sym(A) = (A + A^T)/2.
 *   - Plain lhaf: A's diagonal is ignored; gamma gives the loop weights.
 *   - Repeated form lhaf(A_r): row/column i is repeated r_i times; two copies
 *     of mode i couple with A_ii; every copy has loop weight gamma_i (App. A,
 *     construction of A_n).
 *   - N = sum of sizes (or of r); odd N is padded with one vertex that has no
 *     couplings and loop weight 1, which leaves the value unchanged.
 *   - Limits: N <= 64 per problem.
 *
 * Ownership and errors
 *   - Every pointer belongs to the caller.  Device pointers must stay valid
 *     until the work queued on `stream` has finished.  Host pointers (r,
 *     idx_off, opts) are read before the call returns.
 *   - Arguments are validated synchronously; a non-zero status means nothing
 *     was queued.  Results are valid after the stream is synchronised.
 *   - A non-finite entry that a problem reads (its matrix entries off the
 *     diagonal, its loop weights; for repeated problems also A_ii) or an
 *     overflow gives a NaN result and err_est = +Inf for that problem only.
 *   - The library keeps no state except one lazily created scratch buffer per
 *     device (used when opts->workspace is NULL) and the schedule cache read
 *     from $LHAF_TUNE_CACHE.  Calls on different streams of one device must
 *     pass their own workspaces.
 */
#ifndef LHAF_H
#define LHAF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} lh_c128;

typedef int32_t lh_status;
#define LH_OK 0
#define LH_EINVAL 1        /* bad argument (null pointer, negative size ...) */
#define LH_ESIZE 2         /* problem too large (N > 64) */
#define LH_EHIP 3          /* a HIP runtime call failed */
#define LH_ENOMEM 4        /* workspace too small / allocation failed */
#define LH_EUNSUPPORTED 5  /* option combination not supported */
#define LH_ESCRATCH 6      /* batch too large for lhaf_batched_noalloc's fixed scratch */

#define LH_SUM_ET 0  /* eigenvalue-trace inclusion/exclusion (App. B.1/B.2) */
#define LH_SUM_FDS 1 /* finite-difference sieve (App. B.4), sign-halved */
#define LH_ACC_FP64 0 /* plain double accumulation of the signed term sum */
#define LH_ACC_DD 1   /* double-double (TwoProd/TwoSum) accumulation */
/* LH_ACC_DD_COMP: double-double accumulation, and every term's characteristic
   polynomial (the cofactor recurrence on its Hessenberg form) and the two
   power-series recurrences kept in double-double: each new value is a
   compensated dot product of double-double operands (TwoProd / TwoSum,
   Ogita, Rump and Oishi 2005) stored unrounded, and the final lambda^n
   coefficient is formed the same way and rounded once.  The Hessenberg
   reduction and the loop moments stay FP64.  Per-term errors of
   ill-conditioned terms drop by about two orders of magnitude; a term costs
   1.4x to 1.8x as much (N = 52 .. 40).  Values only: lhaf, lhaf_repeated,
   lhaf_batched (not fused, no saved), lhaf_batched_noalloc and lhaf_mixed;
   the other entry points return LH_EUNSUPPORTED.  err_est is the same
   a-priori estimate as for LH_ACC_DD. */
#define LH_ACC_DD_COMP 2

typedef struct {
  int32_t sum;        /* LH_SUM_FDS (default) or LH_SUM_ET */
  int32_t acc;        /* LH_ACC_DD (default), LH_ACC_FP64 or LH_ACC_DD_COMP */
  int64_t term_begin; /* first term of the enumeration to include (default 0) */
  int64_t term_end;   /* one past the last term, -1 = all (default) */
  int32_t scaled;     /* 1 (default): out = lhaf.  0: out = raw partial sum over
                         [term_begin, term_end) without the 2^-n FDS prefactor,
                         for splitting one lhaf across calls or devices */
  int32_t schedule;   /* -1 (default): tuned/heuristic; >= 0: index into the
                         schedule table (lhaf_schedule_count()) */
  void* workspace;    /* device scratch; NULL = library-owned buffer */
  size_t ws_bytes;
  lh_c128* out_lo;    /* nullable device array: low parts of the double-double
                         results (out holds the high parts) */
  lh_c128* saved;     /* nullable device array of lhaf_saved_count() per-term
                         series coefficients shared by one lhaf_batched call and
                         the lhaf_backward call on the same batch, sum mode and
                         term range: the forward writes a_k = e_{n-k}/2
                         (k = 1..n, e_j the lambda^j coefficient of
                         exp(sum_k g_k lambda^k)) of every term of the range,
                         the backward reads them instead of repeating the
                         Hessenberg reduction.  Problem b's block starts after
                         the blocks of problems < b; term t's entries start at
                         (t - term_begin_b) * n_b inside it, term_begin_b being
                         the range clipped to the problem.  The backward trusts
                         the contents. */
  int64_t saved_count; /* entries available at saved */
  lh_c128* grads;     /* nullable device array of lhaf_grads_count() entries:
                         the per-problem reduced gradient of a batch (LD^2 + 64
                         entries per problem, LD = 8 ceil(m/8)).  On
                         lhaf_batched / lhaf / lhaf_repeated it selects the
                         fused pass: one persistent launch evaluates every term
                         once, adds c_t f_t into the values (out, err_est,
                         opts->scaled honoured) and the term's adjoint into
                         grads (with the FDS prefactor; a term range gives its
                         share).  On lhaf_backward over the same batch it
                         replaces the term pass: only the mapping to dA,
                         dgamma with grad_out runs.  Nothing per term is kept.
                         Not with saved, nor with the other entry points. */
  int64_t grads_count; /* entries available at grads */
} lh_opts;

/* Term enumeration (identical for every entry point).  Pairs p = 0..H-1 with
 * repeat counts eta_p, n = sum eta_p.  A term is a mixed-radix number, pair 0
 * the fastest digit s_p:
 *   ET : radix eta_p + 1; weight z_p = s_p; coefficient
 *        (-1)^(n - sum s) prod C(eta_p, s_p); the all-zero term is 0.
 *   FDS: the halving pair hp is the first pair with odd eta (else pair 0),
 *        radix floor(eta_hp/2) + 1; other pairs radix eta_p + 1; weight
 *        d_p = eta_p - 2 s_p; coefficient prod (-1)^(s_p) C(eta_p, s_p), times 2
 *        for the halving pair unless 2 s_hp = eta_hp; prefactor 2^-n.
 * Plain problems pair position i with position N/2 + i (eta = 1).  Repeated
 * problems use the greedy matching (sort by count descending, ties by index
 * ascending; (m1,m1) x floor(n1/2) if n1 >= 2 n2, else (m1,m2) x n2).
 */

void lh_opts_default(lh_opts* opts);
const char* lh_status_string(lh_status s);
int32_t lhaf_schedule_count(void);

/* Number of terms of the enumeration for one problem (host only, no GPU).
 * r: host multiplicities (NULL = plain problem of size N). */
int64_t lhaf_term_count(int32_t N, const int32_t* r, int32_t sum);

/* Host planner output for one problem (for inspection and tests).
 * pos: 2H entries, pos[p] and pos[H+p] are the two ends of pair p as indices
 * into the problem's index list (-1 = padding vertex); eta: H repeat counts.
 * Returns H, or a negative lh_status. */
int32_t lhaf_plan_pairs(int32_t N, const int32_t* r, int32_t* pos, int32_t* eta);

/* lhaf(A, gamma) of one N x N matrix (App. B).
 * A: device, N x N, row-major, leading dimension lda >= N; diagonal ignored.
 * gamma: device, N loop weights.  out: device, 1 value.  err_est: device,
 * nullable, absolute error estimate of out.  N = 0 gives 1. */
lh_status lhaf(const lh_c128* A, int64_t lda, const lh_c128* gamma, int32_t N, lh_c128* out,
               double* err_est, const lh_opts* opts, void* stream);

/* lhaf(A_r, gamma_r): row/column i of the M x M matrix A repeated r_i times
 * (App. A; the collision form of App. B.2/B.3).  r: HOST, M entries >= 0,
 * sum r <= 64.  r = all ones equals lhaf on A. */
lh_status lhaf_repeated(const lh_c128* A, int64_t lda, const lh_c128* gamma, const int32_t* r,
                        int32_t M, lh_c128* out, double* err_est, const lh_opts* opts,
                        void* stream);

/* Many loop hafnians in one persistent launch (App. B.5 batching; the
 * chain-rule step of App. A.2 needs many lhafs of different sizes).
 * Problem b uses the matrix A_base + b*stride_A (stride_A = 0: one shared
 * base matrix) and gamma_base + b*stride_g, restricted to the index list
 * idx[idx_off[b] .. idx_off[b+1]) (idx: device, NULL = 0,1,2,...);
 * idx_off: HOST, B+1 entries.  r: HOST, nullable, multiplicities packed like
 * idx (NULL = plain).  out: device [B]; err_est: device [B] or NULL.
 * workspace: device, at least lhaf_batched_workspace(...) bytes. */
size_t lhaf_batched_workspace(int32_t B, const int64_t* idx_off, const int32_t* r,
                              const lh_opts* opts);
lh_status lhaf_batched(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                       const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                       const int64_t* idx_off, const int32_t* r, lh_c128* out, double* err_est,
                       void* workspace, size_t ws_bytes, const lh_opts* opts, void* stream);

/* lhaf_batched for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same problems, options, results and errors as lhaf_batched, with the
 * workspace taken from a fixed device array inside the library instead of
 * one the caller passes (opts->workspace is ignored).  The call makes no
 * hipMalloc, hipFree, pinned-host or other device allocation; the plan
 * tables are copied from pageable host memory.  The array holds
 * lhaf_noalloc_scratch_bytes() bytes (64 MiB) on every GPU the library runs
 * on, until the process ends; a batch whose workspace (lhaf_batched_workspace)
 * exceeds it returns LH_ESCRATCH and queues nothing.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams or
 * host threads, before the previous call's work has finished) race and give
 * wrong results.  Calls queued one after another on the same stream are safe.
 * The caller still owns A_base, gamma_base, idx, out, err_est and any
 * opts->out_lo / opts->saved. */
lh_status lhaf_batched_noalloc(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                               const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                               const int64_t* idx_off, const int32_t* r, lh_c128* out,
                               double* err_est, const lh_opts* opts, void* stream);
size_t lhaf_noalloc_scratch_bytes(void);

/* Mixed-state form lhafmix(A, gamma, n) (App. B.2): A is 2M x 2M (device,
 * lda >= 2M), gamma has 2M entries, n (HOST, M entries >= 0) gives the photon
 * numbers; row i and row M+i are both repeated n_i times and paired with each
 * other n_i times, so the sum has prod(n_i + 1) terms (ET) and pairs with
 * n_i = 0 are dropped.  Equals lhaf_repeated on A with r = (n, n);
 * 2 sum(n) <= 64.  Plain term ranges, the coefficient store and error
 * estimates work as for lhaf. */
lh_status lhaf_mixed(const lh_c128* A, int64_t lda, const lh_c128* gamma, const int32_t* n,
                     int32_t M, lh_c128* out, double* err_est, const lh_opts* opts, void* stream);

/* lhaf of a real symmetric matrix with real loop weights (e.g. the
 * non-negative matrices of the MIS independence proposal, App. C), in real
 * FP64 arithmetic: the same sums, enumeration and coefficients as lhaf /
 * lhaf_repeated (r: HOST multiplicities or NULL = plain M x M).  A, gamma:
 * device doubles (lda >= M); out, err_est (nullable): device, one double.
 * opts->saved and opts->out_lo are not supported (LH_EUNSUPPORTED). */
lh_status lhaf_real(const double* A, int64_t lda, const double* gamma, const int32_t* r,
                    int32_t M, double* out, double* err_est, const lh_opts* opts, void* stream);

/* One chain-rule step (App. B.5, batching over the batched mode's outcome):
 * out[k] = lhaf(A_{r(k)}, gamma_{r(k)}), k = 0..n_cut, where r(k) is the host
 * pattern r (M entries, r[mode_b] must be 0) with mode_b set to k photons.
 * One pass over the ET terms of the largest pattern (mode_b paired with
 * itself floor(n_cut/2) times and once with a padding vertex) serves every
 * output: the power traces are shared, each output takes its own binomial
 * weights and lambda degree.  Requires opts->sum = LH_SUM_ET (else
 * LH_EUNSUPPORTED); sum(r) + n_cut <= 64 and n_cut <= 63.  A, gamma: device,
 * M x M (lda) and M; out: device [n_cut+1]; err_est: device [n_cut+1] or NULL.
 * opts->workspace, if set, needs at least the bytes of the equivalent
 * lhaf_repeated call plus (n_cut+1) partials per work item; NULL uses the
 * library buffer. */
lh_status lhaf_chain(const lh_c128* A, int64_t lda, const lh_c128* gamma, const int32_t* r,
                     int32_t M, int32_t mode_b, int32_t n_cut, lh_c128* out, double* err_est,
                     const lh_opts* opts, void* stream);

/* Sub-detector batching (App. B.5): out[g] = lhaf(A_r, gamma_g) for G loop
 * weight vectors gamma_g = gammas + g*ldg (device, M entries each) of one
 * matrix (r: HOST multiplicities or NULL = plain M x M).  The Hessenberg and
 * characteristic-polynomial work of each term is done once; the loop moments
 * and exponential series once per vector.  ET or FDS; 1 <= G <= 64.
 * out, err_est: device [G]. */
lh_status lhaf_gammas(const lh_c128* A, int64_t lda, const lh_c128* gammas, int64_t ldg,
                      const int32_t* r, int32_t M, int32_t G, lh_c128* out, double* err_est,
                      const lh_opts* opts, void* stream);

/* Entries (lh_c128) of the per-term coefficient store of the batch for
 * opts->sum and opts' term range: sum over problems of (terms in the range)
 * x n.  Host only; a negative value is -lh_status. */
int64_t lhaf_saved_count(int32_t B, const int64_t* idx_off, const int32_t* r, const lh_opts* opts);

/* Gradients of the batch above (the paper has none; adjoint of the per-term
 * power-trace recursion).  Holomorphic derivative, returned in PyTorch's
 * convention for complex inputs:
 *   dA_b = grad_out_b * conj(d lhaf_b / d A_b),  dgamma likewise,
 * where lhaf is read as a function of the full matrix through sym(A), so
 *   d lhaf / d A_ij = d lhaf / d A_ji = lhaf(A without rows/cols i,j) / 2  (i != j),
 *   d lhaf / d gamma_i = lhaf(A without row/col i),
 *   d lhaf / d A_ii = 0 for plain problems, C(r_i,2) lhaf(A_{r-2e_i}) repeated.
 * base_dim: rows of each matrix (1..4096; lda >= base_dim); every index list
 * entry must be below it.  dA: device; if stride_A != 0, problem b writes the
 * base_dim x base_dim block dA + b*stride_A (lda) and dgamma + b*stride_g
 * (base_dim entries), rows no vertex maps to getting 0; if stride_A == 0,
 * gradients of all problems are summed into one base-sized dA and dgamma.
 * Both are overwritten (not accumulated).
 * opts->term_begin / term_end select a term range of every problem: the
 * result is that range's share of the gradient (FDS prefactor applied), so
 * the results of disjoint ranges covering all terms add up to the full
 * gradient (each term is independent, App. B.6).  opts->scaled is ignored.
 * With opts->saved, the store must come from the forward over the same
 * batch, sum mode and term range.
 * workspace: at least lhaf_backward_workspace(...) bytes. */
size_t lhaf_backward_workspace(int32_t B, const int64_t* idx_off, const int32_t* r,
                               int32_t base_dim, const lh_opts* opts);
/* Entries (lh_c128) of opts->grads for the batch (host only; negative:
 * -lh_status). */
int64_t lhaf_grads_count(int32_t B, const int64_t* idx_off, const int32_t* r);
lh_status lhaf_backward(int32_t B, const lh_c128* A_base, int64_t lda, int64_t stride_A,
                        const lh_c128* gamma_base, int64_t stride_g, const int32_t* idx,
                        const int64_t* idx_off, const int32_t* r, const lh_c128* grad_out,
                        lh_c128* dA, lh_c128* dgamma, int32_t base_dim, void* workspace,
                        size_t ws_bytes, const lh_opts* opts, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LHAF_H */
