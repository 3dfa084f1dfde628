/* mvn.h - C ABI of the MI355X (gfx950) separation-of-variables MVN library.
 *
 * Computes Phi_n(a, b; mu, Sigma) = P(a <= X <= b), X ~ N(mu, Sigma)
 * (arXiv 2405.14892, Section III-A, Eq. (q1)) with Genz's separation of
 * variables (Section III-B, Eqs. (sov1)-(sov2)) over randomised Richtmyer
 * quasi-Monte Carlo points, organised as the paper's PMVN/QMC algorithms
 * (Algorithms 2 and 3) but as one persistent GPU sweep per sample block.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* or documented "device" are device (HBM) pointers;
 *     all others are host pointers.  The library never allocates device
 *     memory: callers size buffers with the *_bytes queries and pass them in.
 *   - Calls are asynchronous on the given stream and return after host-side
 *     validation and enqueue, except where an entry point's comment says it
 *     synchronises the stream.  Results are ready when the stream reaches them.
 *   - Return value 0 = enqueued.  A negative value -k means argument k
 *     (1-based) is invalid; nothing was enqueued.  -1000 - e means a HIP
 *     runtime error e at launch.  mvn_last_error() gives a message.
 *   - Matrices are row-major; Sigma is symmetric so only its lower triangle
 *     is read and row- or column-major storage are equivalent.
 *   - Only one call per stream at a time uses a given workspace.
 */
#ifndef MVN_H
#define MVN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the Cholesky trailing updates and the SOV limit-update GEMMs
 * (MFMA; FP32 accumulation for the reduced types).  The diagonal-block
 * factorisation and panel solves, the in-block recurrence, log and the
 * per-sample log-products are always FP64.  Phi and Phi^-1 of the
 * conditioning step are FP64 in MVN_FP64; in the reduced modes they run in
 * FP32 where both conditional limits are >= -5 and the interval mass keeps
 * at least half of Phi(b') (log d and y within a few 1e-6), FP64 elsewhere.
 *   MVN_BF16X3: operands split as x = hi + lo (both BF16) and the products
 *   hi*hi + hi*lo + lo*hi accumulated (about 16 significant bits). */
typedef enum { MVN_FP64 = 0, MVN_FP32 = 1, MVN_BF16 = 2, MVN_BF16X3 = 3 } mvn_precision;

/* Trailing-update arithmetic of a dense factorisation whose precision is
 * not MVN_FP64 (the sweep's GEMM always uses `precision`; the paper names
 * mixed precision for these updates as future work, Section VII).
 *   MVN_CHOL_ADAPTIVE (default): a tile-wise precision map.  The update of
 *     trailing tile (i, j) by tile column k, L_ik L_jk^T, runs in the reduced
 *     type when its rounding-error bound u ||L_ik||_F ||L_jk||_F (u: the
 *     type's unit roundoff plus K 2^-24 for FP32 accumulation over the
 *     tile's K products) is at most chol_tol * max_i Sigma_ii, otherwise in
 *     FP32 when FP32's bound is, otherwise in FP64.  Tiles next to the
 *     diagonal, whose panel blocks carry the factor's mass, stay precise.
 *   MVN_CHOL_UNIFORM: every trailing update in the reduced type (loses
 *     positive definiteness on ill-conditioned Sigma: a BF16 factorisation of
 *     a Matern 3/2 field on a 128 x 128 grid with condition number about 4e6
 *     fails at pivot 517).
 *   MVN_CHOL_FP64: the factorisation in FP64; the reduced type is used only
 *     by the sweep's limit-update GEMM. */
typedef enum { MVN_CHOL_ADAPTIVE = 0, MVN_CHOL_UNIFORM = 1, MVN_CHOL_FP64 = 2 } mvn_chol_mode;

/* Matern covariance parameters (Section IV-A, Eq. for C(h; theta)):
 * C(h) = sigma2 / (2^(nu-1) Gamma(nu)) (h/beta)^nu K_nu(h/beta), plus
 * nugget on the diagonal.  The paper calls the range "a"; here it is beta.
 * Any 0 < nu <= 20: nu = 0.5, 1.5, 2.5 by the closed forms of K_nu at
 * half-integer order; other nu by the trapezoidal rule on the integral
 * K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, relative accuracy about
 * 1e-14 (up to 1e-13 where the result is below 1e-250).  Other values are
 * rejected with the position of the kernel argument. */
typedef struct mvn_matern {
  double sigma2, beta, nu, nugget;
} mvn_matern;

typedef struct mvn_options {
  int tile;          /* Cholesky tile size m (Algorithm 1).  Dense: >= 16 and  */
                     /* a multiple of 4.  TLR: a multiple of 128 in           */
                     /* [128, 1024]                                           */
  int precision;     /* mvn_precision (TLR factors: MVN_FP64 only)            */
  int periodize;     /* 1 = baker's transform of the QMC points, 0 = off       */
  int sweep_rows;    /* rows per block of the dense, batched and TLR sweeps:  */
                     /* 128 (two workgroups per CU) or 64 (four, three for   */
                     /* split BF16: more sample columns conditioned at once, */
                     /* Y read twice as often); 0 = 128 for dense factors    */
                     /* and batches, 64 for TLR factors, which also take     */
                     /* 256: 256 sample columns per workgroup, each wave     */
                     /* conditioning its own 64 (64-row blocks; on request   */
                     /* only).  The adjoint sweep                            */
                     /* uses 128.  32 (dense FP64 mvn_prob, mvn_prob_prefix, */
                     /* mvn_prob_static): the narrow sweep, 16 sample        */
                     /* columns per workgroup (32 above 20480 samples), the  */
                     /* next block's GEMM overlapped with the recurrence;    */
                     /* 0 selects it for dense FP64 calls with N*S <= 20480  */
                     /* and N*S*n <= 9e7 (4.5e7 above 12288 samples, where  */
                     /* the chunks are 32 columns wide)                      */
  double tlr_eps;    /* > 0: tile low-rank factor (Section III-E): every      */
                     /* off-diagonal tile is compressed to U V^T with         */
                     /* ||A_ij - U V^T||_F <= tlr_eps (absolute).  <= 0: dense */
  int max_rank;      /* TLR rank cap, 1 .. min(256, tile)                      */
  int chol_mode;     /* mvn_chol_mode (dense factors, precision != MVN_FP64)   */
  double chol_tol;   /* MVN_CHOL_ADAPTIVE: error bound per tile update,        */
                     /* relative to max_i Sigma_ii; <= 0 selects 1e-9          */
} mvn_options;

/* Factor handle, filled by mvn_cholesky.  Plain data; copy freely.
 * opts->precision selects the trailing-update arithmetic and which operand
 * copy of L is kept for the sweep.  *info (device int) is 0 on success or
 * k > 0 if the leading minor of order k is not positive definite (LAPACK
 * dpotrf convention), or -1 if the site permutation of
 * mvn_cholesky_permuted was not a permutation.
 *
 * Dense factor (flags == 0): L is row-major with leading dimension ld (>= n,
 * a multiple of 128); rows and columns n..ld-1 hold the identity so blocked
 * kernels need no bounds checks.
 *
 * Tile low-rank factor (flags & MVN_FACTOR_TLR), tile edge m = tile,
 * nt = ld / m tiles per side, rank stride rs = max_rank rounded up to 16:
 *   L      the nt(nt+1)/2 lower m x m tiles, tile (i, j) at
 *          (i(i+1)/2 + j) m^2 doubles, row-major with leading dimension m.
 *          Diagonal tiles hold the dense factors L_ii; off-diagonal tiles
 *          hold the updated covariance tiles they were compressed from.
 *   U, Vt  for i > k, panel p = i(i-1)/2 + k: U at p m rs doubles (m x rs,
 *          row-major), Vt at p rs m doubles (rs x m, row-major), with
 *          L_ik = U_ik Vt_ik (columns / rows past the rank are zero).
 *   ranks  device int per panel; negative when max_rank stopped the
 *          compression before the residual reached tlr_eps. */
#define MVN_FACTOR_TLR 1
/* Compact TLR factor (flags == MVN_FACTOR_TLR | MVN_FACTOR_TLR_COMPACT, from
 * mvn_tlr_compact): only what the sweep reads, at the actual ranks.
 *   L      the nt diagonal tiles, tile i at i m^2 doubles (row-major, m)
 *   Vt     the V'^T rows of every panel (i, j), i > j, stacked by tile
 *          column j in order of i (sum of the ranks rows of m doubles), then
 *          128 zero rows
 *   U      per tile-row i the U columns of its panels side by side (m rows
 *          of Kpad_i doubles, Kpad_i = the sum of the row's ranks rounded up
 *          to 16, zero columns past it), tile-rows one after another
 *   ranks  as above (a copy) */
#define MVN_FACTOR_TLR_COMPACT 2
typedef struct mvn_factor {
  int n;
  int ld;           /* dense: padded n; TLR: nt * tile                         */
  int precision;    /* arithmetic the factor was built with (mvn_precision)    */
  int flags;        /* 0, MVN_FACTOR_TLR, or MVN_FACTOR_TLR | ..._COMPACT     */
  double* L;        /* device: dense ld*ld doubles, or the TLR tiles           */
  int* info;        /* device, 1 int                                           */
  void* L_low;      /* device copy of L as the sweep's GEMM operand: ld*ld     */
                    /* floats (FP32), BF16 (BF16), two BF16 planes (BF16X3);  */
                    /* NULL for FP64 and TLR                                   */
  int tile;         /* TLR tile edge m (0 for dense)                           */
  int rank_stride;  /* TLR rs (0 for dense)                                    */
  double* U;        /* device, TLR only                                        */
  double* Vt;       /* device, TLR only                                        */
  int* ranks;       /* device, TLR only                                        */
  double tlr_eps;   /* TLR accuracy the factor was built with                  */
  int max_rank;     /* TLR rank cap                                            */
  int chol_mode;    /* mvn_chol_mode the dense factor was built with           */
  unsigned long long* update_counts;  /* device, 3 counters (dense factors):   */
                    /* trailing tile updates run in FP64, FP32 and the reduced */
                    /* type by the adaptive map (all zero in the other modes)  */
} mvn_factor;

/* Sizes.  All return 0 on success and write the byte count.
 * mvn_prob_workspace_bytes with TLR options (tlr_eps > 0) returns a size
 * that holds any factor built with those options (every tile at the rank
 * stride), usually far more than needed; mvn_prob_workspace_bytes_factor
 * returns the size for a given factor: for a TLR factor it reads the ranks
 * back, which synchronises `stream` (the stream the factor was built on;
 * query once, outside any graph capture); for a dense factor it equals mvn_prob_workspace_bytes(f->n, ...) and does
 * not touch the device.  With a smaller TLR workspace mvn_prob runs as many
 * persistent sweep workgroups as fit (slower, same result). */
int mvn_factor_bytes(int n, const mvn_options* opts, size_t* bytes);
int mvn_cholesky_workspace_bytes(int n, const mvn_options* opts, size_t* bytes);
int mvn_prob_workspace_bytes(int n, int N, int S, const mvn_options* opts, size_t* bytes);

/* Sigma = L L^T (Algorithm 1, covariance generation and factorisation).
 * With opts->tlr_eps > 0 the factor is tile low-rank (Section III-E): the
 * tiles are factored right-looking; each off-diagonal panel tile is
 * compressed by adaptive cross approximation, accepted only when the exact
 * residual Frobenius norm is <= tlr_eps, then L_ik = U_ik (L_kk^{-1} V_ik)^T
 * and the trailing tiles are updated with the low-rank products (FP64).
 * The TLR factorisation needs the workspace of
 * mvn_cholesky_workspace_bytes; the dense one needs none.
 *   n        dimension (>= 1)
 *   d_sigma  device n x n covariance with row stride ld_sigma, or NULL to
 *            generate it from d_locs and kern (Matern + nugget)
 *   d_locs   device n x 2 locations (x, y), read when d_sigma is NULL
 *   factor_buf / factor_bytes   device memory for the factor
 *   ws / ws_bytes               device workspace (may be NULL if 0 bytes)
 *   out      host struct receiving the handle
 * Non-positive-definite input is reported in *out->info (device), not by
 * the return value; later kernels on the stream see it and propagate NaN. */
int mvn_cholesky(int n, const double* d_sigma, int ld_sigma, const double* d_locs,
                 const mvn_matern* kern, const mvn_options* opts,
                 void* factor_buf, size_t factor_bytes, void* ws, size_t ws_bytes,
                 mvn_factor* out, hipStream_t stream);

/* P(a <= X <= b) by the SOV estimator (Algorithm 2 with Eq. (sov1)), over
 * N Richtmyer points j = 1..N and S random shifts drawn from `seed`.
 *   d_a, d_b  device limits (n doubles, may be -inf / +inf, a_i <= b_i)
 *   d_mu      device mean (n doubles) or NULL for a zero mean
 *   d_out     device output, 4 + S doubles:
 *               [0] log P-hat  [1] P-hat (0 on underflow)
 *               [2] standard error of P-hat over shifts (NaN if S == 1)
 *               [3] relative standard error   [4 + s] log P-hat of shift s
 *             All NaN if the factor's info != 0 or a limit is NaN / a > b.
 *   d_ell     device, N*S doubles or NULL: per-sample log prod d_i, sample
 *             column c = s*N + (j-1).
 * opts->precision selects the arithmetic of the limit-update GEMM: MVN_FP64
 * always, or the precision the factor was built with.  For a TLR factor
 * (FP64 only) the update of tile-row i is sum_j U_ij (Vt_ij Y_j) plus the
 * dense diagonal tile: once the samples of tile j are known, Vt_ij Y_j is
 * formed for all i > j in one stacked product, and the update of tile-row i
 * is one product with the ranks packed along K.  The index tables of those
 * products and the layout of the rank-dependent part of the workspace are
 * built on the device from the factor's ranks, so the call reads nothing
 * back and can be captured in a graph.  Its workspace size comes from
 * mvn_prob_workspace_bytes_factor (which reads the ranks back) or the TLR
 * bound of mvn_prob_workspace_bytes; the sweep runs as many persistent
 * workgroups as the workspace holds for the actual ranks.  A workspace below
 * the size of the rank-independent part plus one workgroup at rank zero is
 * rejected (-10); one that holds no workgroup for the actual ranks gives NaN
 * outputs.
 * The QMC point of sample (s, j) in dimension i is
 *   w = ((j*A_i + D_{s,i} mod 2^64) >> 11 + 1/2) 2^-53 with
 *   A_i = floor(frac(sqrt(p_{i+1})) 2^64) (p_k the k-th prime) and
 *   D_{s,i} = SplitMix64 output s*n + i from state `seed`. */
int mvn_prob(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu,
             int N, int S, uint64_t seed, const mvn_options* opts,
             void* ws, size_t ws_bytes, double* d_out, double* d_ell, hipStream_t stream);

int mvn_prob_workspace_bytes_factor(const mvn_factor* f, int N, int S, const mvn_options* opts,
                                    size_t* bytes, hipStream_t stream);

/* mvn_prob for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same estimator, arguments and outputs as mvn_prob, with the
 * workspace taken from a 256 MiB device array inside the library instead of
 * a caller buffer.  Each GPU the library runs on holds its own copy of the
 * array until the process ends; the first call on a device looks up its
 * address and copies the QMC lattice table into it (a synchronous copy), and
 * later calls only enqueue kernels.  Nothing is allocated.
 *   Dense factors only (any precision the factor holds), n <= 131072.  The
 *   sweep runs as many persistent workgroups as the array holds (fewer than
 *   mvn_prob for large n: slower, same result); a problem whose single
 *   workgroup does not fit (about n * (1 KiB + 24 B) + 8 N S bytes with
 *   d_ell == NULL) is rejected with -5.
 *   Every call on one GPU shares that GPU's array: calls that overlap on one
 *   GPU (different streams, or threads) race and must be serialised by the
 *   caller.  Each call writes every scratch entry it reads, so no clearing
 *   is needed between calls. */
int mvn_prob_static(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu,
                    int N, int S, uint64_t seed, const mvn_options* opts, double* d_out,
                    double* d_ell, hipStream_t stream);

/* Nested-set probabilities of confidence-region detection (Section III-C with
 * Algorithm 1 of Section IV-A), for the sites in the factor's order (the caller orders them,
 * e.g. by decreasing marginal exceedance probability, before building the
 * factor): log P-hat(a_i <= X_i <= b_i, i < k) for every k = 1..n from ONE
 * sweep.  The running product d_1 .. d_k of every sample is a sample of the
 * k-site problem, because the leading k x k block of L is the Cholesky factor
 * of the leading block of Sigma; the sweep records it after every row.  Same
 * estimator, QMC points and limits as mvn_prob (the last entry is mvn_prob's
 * log P-hat up to rounding), so P-hat of the first k sites uses the n-site
 * problem's points for its k dimensions.
 *   N         >= 64 (a chunk of 64 consecutive samples then meets at most two
 *             shifts)
 *   d_prefix  device, 2n doubles: [2(k-1)] log P-hat of the first k sites,
 *             [2(k-1) + 1] its relative standard error over the shifts (NaN
 *             if S == 1).  All NaN if the factor's info != 0 or a limit is
 *             NaN / a > b.
 * Dense factors (any precision the factor holds) and TLR factors (FP64), as
 * for mvn_prob.  The workspace holds n x ceil(N S / 64) x 4 + n S doubles,
 * then mvn_prob's; mvn_prob_prefix_workspace_bytes gives its size for the
 * factor (for a TLR factor it reads the ranks back, synchronising `stream`;
 * mvn_prob_prefix itself does not). */
int mvn_prob_prefix_workspace_bytes(const mvn_factor* f, int N, int S, const mvn_options* opts, size_t* bytes,
                                    hipStream_t stream);
int mvn_prob_prefix(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu,
                    int N, int S, uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes,
                    double* d_prefix, hipStream_t stream);

/* The site order of Algorithm 1 (Section IV-A) for confidence-region
 * detection: sites by decreasing marginal exceedance probability
 * p_i = Phi((mu_i - u) / sqrt(var_i)), ties by increasing site index (a
 * variance <= 0 gives p_i = 1 if mu_i > u, else 0).  For a posterior the
 * inputs are mvn_posterior's mu_post and var_post, and d_perm goes straight
 * to mvn_cholesky_permuted, so the workflow never reads back.
 *   d_mu, d_var  device, n doubles
 *   d_perm       device output, n int64 site indices; all -1 if a variance
 *                is NaN or a mean is not finite
 *   d_p          device output, n doubles (p_i in site order), or NULL
 *   ws           device workspace of mvn_exceedance_order_workspace_bytes
 *                (16 bytes per element of the next power of two >= n)
 * A bitonic sort on the device; asynchronous on `stream`. */
int mvn_exceedance_order_workspace_bytes(int n, size_t* bytes);
int mvn_exceedance_order(int n, const double* d_mu, const double* d_var, double u, int64_t* d_perm, double* d_p,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* A TLR factor with its storage cut to the ranks (the representation of
 * Section III-E keeps only the diagonal tiles and the low-rank factors):
 * the diagonal tiles and U, V'^T packed at the actual ranks in the order the
 * sweep reads them (layout at MVN_FACTOR_TLR_COMPACT), about 2 m^2 per tile
 * column plus 16 m bytes per unit of rank instead of nt(nt+1)/2 dense tiles
 * and U, V'^T at the rank stride.  mvn_prob and mvn_prob_prefix accept the
 * compact factor and give bit-identical results (they read the packed
 * factors directly instead of packing them per call); mvn_tlr_dense does
 * not take it.  Both calls read the ranks back, which synchronises `stream`
 * (a one-time step after the factorisation); *out shares nothing with f,
 * whose buffer may then be freed.
 *   d_buf / bytes   device memory, at least mvn_tlr_compact_bytes */
int mvn_tlr_compact_bytes(const mvn_factor* f, size_t* bytes, hipStream_t stream);
int mvn_tlr_compact(const mvn_factor* f, void* d_buf, size_t bytes, mvn_factor* out, hipStream_t stream);

/* The TLR factor in dense form: the configuration of Section IV-C, where
 * the factorisation is tile low-rank (Section III-E) and the SOV sweep of
 * Algorithm 2 runs on dense tiles.  Writes L into d_buf as a dense FP64
 * factor, row-major with leading dimension ld = n rounded up to 128:
 * diagonal tiles copied, off-diagonal tiles L_ij = U_ij V'^T_ij (FP64 MFMA),
 * identity past n; the upper triangle is not written (no sweep reads it).
 * *out receives a dense FP64 factor handle on d_buf that shares f's info
 * (so a failed TLR factorisation still gives NaN results); it stays valid
 * while d_buf and f's buffer live.  Pass it to mvn_prob / mvn_prob_prefix
 * with a dense workspace (mvn_prob_workspace_bytes with tlr_eps = 0).
 *   d_buf / bytes   device memory, at least mvn_tlr_dense_bytes
 * Returns -1 if f is not a TLR factor, -2 / -3 for a NULL or short buffer,
 * -4 for a NULL out.  Asynchronous on `stream`; nothing is read back. */
int mvn_tlr_dense_bytes(const mvn_factor* f, size_t* bytes);
int mvn_tlr_dense(const mvn_factor* f, void* d_buf, size_t bytes, mvn_factor* out, hipStream_t stream);

/* Factor P Sigma P^T: Sigma given by its lower triangle (device, row stride
 * ld_sigma; the upper triangle is not read), factored in the site order
 * d_perm (device, n int64 entries): row i of the factor is site d_perm[i].
 * This is how a confidence region orders a given Sigma (Algorithm 1: sites
 * by decreasing marginal exceedance probability) before the nested-set
 * sweep.  Options, factor buffer and result as for mvn_cholesky (dense in
 * any precision, or TLR); the workspace is
 * mvn_cholesky_permuted_workspace_bytes (mvn_cholesky's plus n ints and a
 * flag).  d_perm is checked on the device: if it is not a permutation of
 * 0..n-1, *info is -1 and every output computed from the factor is NaN.
 * Asynchronous; nothing is read back. */
int mvn_cholesky_permuted_workspace_bytes(int n, const mvn_options* opts, size_t* bytes);
int mvn_cholesky_permuted(int n, const double* d_sigma, int ld_sigma, const int64_t* d_perm,
                          const mvn_options* opts, void* factor_buf, size_t factor_bytes, void* ws,
                          size_t ws_bytes, mvn_factor* out, hipStream_t stream);

/* Posterior of a Gaussian field x ~ N(mu, Sigma) at n sites, observed at m
 * of them with noise: y = A x + eps, eps ~ N(0, noise_var I), A the m x n
 * indicator matrix of the sites d_obs (Section V-B, the equations for
 * Sigma_post and mu_post, which then replace Sigma and mu in Algorithm 1).
 * Sigma is the Matern covariance of d_locs (n x 2, device) with kern (the
 * nugget is part of Sigma).  Computed as the Woodbury form
 *   Sigma_post = Sigma - C^T K^-1 C,  mu_post = mu + C^T K^-1 (y - mu_o),
 *   K = Sigma_oo + noise_var I,  C = Sigma_o.,
 * by one tiled Cholesky factorisation of the bordered matrix
 * [K C 0; C^T Sigma 0; (y - mu_o)^T 0 1] stopped after the observation
 * columns: its trailing block is Sigma_post and -(mu_post - mu).  FP64.
 *   d_mu         prior mean (n, device) or NULL for zero
 *   d_obs        device, m int64 site indices in 0..n-1; a site may repeat.
 *                Checked on the device: an index out of range gives
 *                *d_info = -1 and NaN outputs
 *   d_y          device, m observations
 *   noise_var    > 0
 *   opts         tile of the factorisation (precision must be FP64)
 *   d_mu_post    device, n (or NULL): posterior mean
 *   d_var_post   device, n (or NULL): posterior marginal variance
 *   d_info       device int: 0, or k > 0 if the k-th leading minor of K is
 *                not positive, or -1 for a bad index (then the outputs are
 *                NaN)
 *   sigma_post   receives a pointer to Sigma_post inside the workspace:
 *                lower triangle, row stride *ld_sigma_post, valid until the
 *                workspace is reused; pass it to mvn_cholesky_permuted
 * Workspace: mvn_posterior_workspace_bytes ((m' + n + 1)^2 doubles, m' = m
 * rounded up to the tile).  Asynchronous; nothing is read back. */
int mvn_posterior_workspace_bytes(int n, int m, const mvn_options* opts, size_t* bytes);
int mvn_posterior(int n, const double* d_locs, const double* d_mu, int m, const int64_t* d_obs,
                  const double* d_y, const mvn_matern* kern, double noise_var, const mvn_options* opts,
                  void* ws, size_t ws_bytes, double* d_mu_post, double* d_var_post, int* d_info,
                  double** sigma_post, int* ld_sigma_post, hipStream_t stream);

/* Monte Carlo check of nested-set probabilities (Section V-C, the check of
 * detected confidence regions by direct sampling): M fields X = mu + L Z
 * from the fitted distribution, for the sites in the factor's order, and for
 * each nested set (the first k sites) the number of fields inside the limits
 * on all of its sites.  Z is standard normal from a counter-based generator:
 *   Z[i, j] = Phi^-1(U),  U = ((SplitMix64 output j n + i from state `seed`)
 *             >> 11) + 1/2) 2^-53          (site i, sample j; 0-based)
 * so a sample can be redrawn on its own.  FP64 (dense factors of any
 * precision: their FP64 L is used).
 *   d_a, d_b  device, n doubles: the limits; the interval is closed, a NaN
 *             limit never holds
 *   d_mu      device mean (n doubles) or NULL for zero
 *   M         >= 1 samples
 *   d_first   device, M ints, or NULL: per sample, the first site (0-based)
 *             with X outside [a, b], n if none; -1 if the factor's info != 0
 *   d_count   device, n int64: [k - 1] = number of samples inside the limits
 *             on the first k sites (= number with first failure >= k);
 *             all -1 if the factor's info != 0
 * A sample is followed only until it fails, and a group of 64 samples stops
 * when all of them have: the work is that of the leading rows of L the
 * samples reach.  opts->sweep_rows: rows per block, 0 = 128, or 64.
 * TLR factors are rejected (-1).  The workspace is
 * mvn_mc_prefix_workspace_bytes; nothing is allocated and the stream is not
 * synchronised.  Returns 0 or a negative argument position. */
int mvn_mc_prefix_workspace_bytes(int n, int M, const mvn_options* opts, size_t* bytes);
int mvn_mc_prefix(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int M,
                  uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes, int* d_first,
                  int64_t* d_count, hipStream_t stream);

/* Gradient of log P-hat at fixed QMC points (the same estimator and points
 * as mvn_prob): reverse-mode differentiation of the recurrence of Eq. (sov1),
 * with checkpointed shifts s_i instead of stored y.  FP64.
 *   d_out            as for mvn_prob (4 + S doubles)
 *   d_da, d_db       device, n doubles each (or NULL): d log P-hat / d a_i,
 *                    d log P-hat / d b_i
 *   d_dmu            device, n doubles (or NULL): d log P-hat / d mu_i =
 *                    -(d/da_i + d/db_i)
 * Infinite limits get a zero derivative.  All outputs NaN under the same
 * conditions as mvn_prob, or when every sample has zero mass.  Dense FP64
 * factors only. */
int mvn_prob_grad_workspace_bytes(int n, int N, int S, const mvn_options* opts, size_t* bytes);
int mvn_prob_grad(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu,
                  int N, int S, uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes,
                  double* d_out, double* d_da, double* d_db, double* d_dmu, hipStream_t stream);

/* ---------------------------------------------------------------- batches
 * Many MVN problems of uneven dimension in one call: the nested sets of
 * confidence-region detection (Algorithm 1 evaluates PMVN on growing
 * subsets of the sites).  Problem p uses the n_p locations
 * d_locs[d_idx[o_p + i]] (o_p = n_0 + ... + n_{p-1}) with the Matern kernel,
 * limits d_a[o_p + i], d_b[o_p + i] and mean d_mu[o_p + i] (or NULL), and the
 * same N, S, seed as mvn_prob for its own dimension.
 *
 * mvn_batch_plan (host only) lays the batch out: it writes `plan`
 * (mvn_batch_plan_bytes(count) bytes of host memory; per-problem offsets and
 * the order of decreasing size) and the factor and workspace sizes.  The
 * caller copies the plan to device memory once and passes it to
 * mvn_prob_batch, whose launch sequence then allocates nothing and never
 * synchronises (it can be captured in a graph and replayed).
 *   n_p     host, count sizes (each >= 1), the same array for both calls
 *   d_idx   device, sum n_p int64 location indices
 *   d_out   device, count x (4 + S) doubles, per problem as for mvn_prob
 *   d_info  device, count ints: Cholesky info per problem
 * The factorisations use 128-wide tiles and opts->precision for the trailing
 * updates and the sweep GEMMs.  Sweep work items (problem, 64 samples) are
 * taken from a device counter in order of decreasing problem size. */
int mvn_batch_plan_bytes(int count, size_t* bytes);
int mvn_batch_plan(int count, const int* n_p, int N, int S, const mvn_options* opts, void* plan,
                   size_t plan_bytes, size_t* factor_bytes, size_t* ws_bytes);
int mvn_prob_batch(int count, const int* n_p, const void* d_plan, const int64_t* d_idx,
                   const double* d_locs, const mvn_matern* kern, const double* d_a, const double* d_b,
                   const double* d_mu, int N, int S, uint64_t seed, const mvn_options* opts,
                   void* factor_buf, size_t factor_bytes, void* ws, size_t ws_bytes, double* d_out,
                   int* d_info, hipStream_t stream);

/* Message for the last negative return on this thread ("" if none). */
const char* mvn_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int mvn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MVN_H */
