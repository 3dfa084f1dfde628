// Host-side launch sequences of the device kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "matern.h"

namespace mvn {

// Lower triangle of the padded ld x ld matrix A (row-major) from the caller's
// Sigma (row stride lds) or from locations with the Matern kernel; rows and
// columns n..ld-1 become the identity.  Also clears *info.
// With perm (device, n entries, checked by launch_index_check, whose flag is
// perm_bad) the matrix is Sigma[perm[i]][perm[j]], read from Sigma's lower
// triangle; a bad permutation gives the identity and *info = -1.
hipError_t launch_build_matrix(int n, int ld, const double* sigma, int lds, const int64_t* perm, const int* perm_bad,
                               const double* locs, const Matern& mk, double* A, int* info, hipStream_t st);

// Device check of an index array: entries in [0, range) and, with `seen`
// (range ints of scratch), no entry twice; *flag = 0 if so, else 1.
hipError_t launch_index_check(const int64_t* idx, long count, long range, int* seen, int* flag, hipStream_t st);

// Zero n 64-bit words with a kernel (not a memset node, so that a caller may
// capture the call in a graph).
hipError_t launch_clear_u64(unsigned long long* p, long n, hipStream_t st);

// A second stream of the current device (default priority, non-blocking)
// with three events, for work that overlaps the caller's stream inside one
// library call.  Created on first use and kept until the process ends; each
// slot is an independent set whose mutex serialises the callers enqueueing
// on it.  nullptr (run everything on the caller's stream) if it cannot be
// created or `st` is being captured into a graph.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ev[3] = {};
  std::mutex mu;
};
constexpr int kSideCholesky = 0, kSideTlr = 1, kSideSlots = 2;
SideStream* side_stream(int slot, hipStream_t st);

// In-place right-looking tiled Cholesky of the padded matrix; *info gets the
// 1-based index of the first non-positive pivot.  Upper triangle zeroed.
// With `lookahead`, the trailing updates off the next tile column run on a
// side stream concurrently with that column's panel factorisation.
// With kstop > 0 (a multiple of tile) only the first kstop columns are
// factored; the trailing block then holds the Schur complement, with every
// update of those columns applied (upper triangle still zeroed).
hipError_t launch_cholesky_f64(int ld, int tile, double* A, int* info, hipStream_t st, bool lookahead = true,
                               int kstop = 0);

// Device state of the adaptive precision map of the mixed factorisation:
// two slots of ld/128 + 1 panel block norms, max diag(Sigma), and the number
// of tile updates run in FP64 / FP32 / the reduced type.
struct LpMap {
  double* norms;
  double* dmax;
  unsigned long long* counts;
  double tol;  // error bound per tile update relative to max diag(Sigma)
};

// The same factorisation with the trailing updates in FP32 (prec 1), BF16
// (2) or split BF16 (3) on MFMA, followed by the low-precision operand copy
// of L for the sweep (`low`: ld*ld floats, ld*ld BF16, or two BF16 planes).
// map != nullptr: each tile update picks FP64, FP32 or the reduced type by
// its rounding-error bound (adaptive precision map); nullptr: every update in
// the reduced type.  fp64_factor: FP64 factorisation, then the copy.
hipError_t launch_cholesky_lp(int prec, int ld, int tile, double* A, int* info, void* low,
                              hipStream_t st, const LpMap* map, bool fp64_factor);

// Monte Carlo check of nested sets: fields X = mu + L Z (dense FP64 factor),
// per sample the first site outside [a, b] (n if none), and per prefix the
// number of samples inside on all of its sites.
struct McArgs {
  const double* L;
  int ld;
  int n;
  const double* a;           // n limits each (device); mu may be nullptr
  const double* b;
  const double* mu;
  uint64_t seed;             // Z[i, j] from SplitMix64 output j n + i of this state
  long M;                    // samples
  double* yscr;              // per-workgroup Z scratch, grid x yslice doubles
  long yslice;               // ld x 64
  int* first;                // M (or nullptr)
  unsigned long long* hist;  // n + 1 bins of first failures (cleared here)
  unsigned long long* counter;  // work-item counter (cleared here)
  long long* count;          // n: samples inside the limits on sites 0..k
  const int* info;           // factor status: != 0 gives first = -1, count = -1
  int grid;                  // workgroups
  int rows;                  // 64 or 128 rows per block
};
int mc_wg_per_cu(int rows);
hipError_t launch_mc(const McArgs& a, hipStream_t st);

// Posterior of a field observed with noise at m sites: the bordered matrix
// [K C 0; C^T Sigma *; r^T 0 1] (ld x ld, lower triangle), factored over its
// first mpad columns (the m observations padded with identity).
struct PosteriorArgs {
  double* B;
  long ld;                 // >= mpad + n + 1, a multiple of 16
  int n, m;
  long mpad;               // m rounded up to the Cholesky tile
  const int64_t* obs;      // m site indices (device)
  const int* obs_bad;      // flag of the device check of obs (out of range: identity, *info = -1)
  const double* locs;      // n x 2
  const double* y;         // m observations
  const double* mu;        // n prior means, or nullptr
  Matern mk;
  double noise_var;
  int* info;               // non-positive pivot of K (1-based), 0 if none
};
hipError_t launch_posterior(const PosteriorArgs& p, int tile, double* mu_post, double* var_post, hipStream_t st);
// Sites by decreasing Phi((mu_i - u) / sqrt(var_i)), ties by index, into perm
// (n entries; all -1 if a variance is not positive or an input is not
// finite); key / idx: npad scratch entries each (npad = the next power of
// two >= n), bad: one int; p_out (n, optional) receives the probabilities.
long exceedance_npad(int n);
hipError_t launch_exceedance_order(int n, const double* mu, const double* var, double u, double* key, int64_t* idx,
                                   int* bad, double* p_out, int64_t* perm, hipStream_t st);

struct SweepArgs {
  const double* L;         // FP64 factor (diagonal blocks, pivots)
  const void* Llow;        // factor in the GEMM's operand type (== L for FP64)
  int ld;
  int n;
  int prec;                // 0 FP64, 1 FP32, 2 BF16, 3 split BF16 (x3)
  const double* at;        // centred lower limits (padded to ld)
  const double* bt;        // centred upper limits
  const uint64_t* lattice; // A_i, n entries
  uint64_t seed;           // shift D_{s,i} = SplitMix64 output s*n + i from this state
  int N, S, periodize;
  void* yscr;              // per-workgroup Y scratch, grid x yslice elements
  long yslice;
  double* ell;             // N*S per-sample log-products
  int grid;                // persistent workgroups
  int rows;                // rows per sweep block: 128 (two workgroups per CU) or 64 (three)
  double* prefix;          // nullptr, or n x nchunks x 4 partials of the running products per row
  int wide;                // FP64, 128 rows, no prefix: the 128-column sweep (yslice = ld x 128)
  int quad;                // the 256-column sweep with four conditioning waves (yslice = quad_yslice)
  int narrow;              // 16 or 32: the FP64 sweep with that many columns per workgroup (yslice = ld x narrow)
};

// Setup of one probability call: centred limits and the invalid-limit flag.
hipError_t launch_prob_setup(int n, int ld, const double* a, const double* b, const double* mu,
                             double* at, double* bt, int* bad, hipStream_t st);

hipError_t launch_sweep(const SweepArgs& a, hipStream_t st);
// The FP64 sweep with 128 sample columns per workgroup (kernels_sov_wide.hip).
hipError_t launch_wide_sweep(const SweepArgs& a, hipStream_t st);
int wide_sweep_cols();
int wide_sweep_wg_per_cu();
// log P-hat of every nested set (first k sites) and its relative standard
// error over shifts from the partials of a prefix sweep: out[2k], out[2k+1].
// cols: sample columns per chunk of the partials (64, or the narrow sweep's 16 / 32).
hipError_t launch_prefix_reduce(const double* part, long nchunks, int cols, int n, int N, int S, double* lps,
                                const int* info_factor, const int* bad_limits, double* out, hipStream_t st);
long sweep_yslice(int prec, int ld);
int sweep_elem_bytes(int prec);

struct GradArgs {
  const double* L;         // FP64 factor (diagonal blocks, pivots, the reverse GEMM)
  const void* Llow;        // forward GEMM operand (== L for FP64; planes ld*ld apart for split BF16)
  int prec;                // forward GEMM arithmetic: 0 FP64, 1 FP32, 2 BF16, 3 split BF16
  int ld;
  int n;
  const double* at;
  const double* bt;
  const uint64_t* lattice;
  uint64_t seed;
  int N, S, periodize;
  double* yscr;    // grid x ld x 64: y of the forward pass
  double* sfw;     // grid x ld x 64: shifts s_i of the forward pass
  double* sbar;    // grid x ld x 64: adjoints of s (reverse pass)
  double* ell;     // N*S per-sample log-products
  double* gpart;   // nchunks x 2 x ld: per-chunk partial gradients (a~, then b~)
  double* mz;      // nchunks x 2: (max l, sum exp(l - max)) per chunk
  int grid;
};

// Forward + adjoint sweep, then the fixed-order combination of the chunks'
// partial gradients into da, db, dmu (each n doubles or NULL).
hipError_t launch_grad(const GradArgs& a, const int* info_factor, const int* bad, double* scale,
                       double* da, double* db, double* dmu, hipStream_t st);

// log-sum-exp over samples, per shift and overall, into out[4 + S].
hipError_t launch_reduce(const double* ell, int N, int S, double* part, const int* info_factor,
                         const int* bad_limits, double* out, hipStream_t st);

int sweep_tile_cols();
// Workgroups of the sweep that share one CU for a block-row count (128 or 64)
// and precision.
int sweep_wg_per_cu(int rows, int prec);

// ---------------------------------------------------------------- batches
// Per-problem descriptor of a batch (written by the host plan, read on the
// device).  Offsets are in elements of the packed buffers.
struct BatchDesc {
  int64_t factor_off;   // L_p at factor + factor_off (ld x ld doubles); low copy at the same offset
  int64_t lim_off;      // limits / location indices of the problem start here
  int64_t tile_off;     // first 64 x 64 lower tile of the problem in the flat build grid
  int32_t n;
  int32_t ld;           // n rounded up to 128
  int64_t reserved;
};
static_assert(sizeof(BatchDesc) == 40, "descriptor layout");

// Sigma_p = C(||s_{idx_i} - s_{idx_j}||) + nugget on the lower tiles of every
// problem (one 64 x 64 tile per workgroup, flat over all problems); clears
// info[p].
hipError_t launch_batch_build(const BatchDesc* desc, int count, long total_tiles, const int64_t* idx,
                              const double* locs, const Matern& mk, double* factor, int* info, hipStream_t st);

// Tiled Cholesky (tile 128) of every problem, one launch per step for all
// problems that still have that step.  ld_rank[r] is the padded size of the
// problem of rank r (ranks sorted by size, largest first); order[r] is its id.
hipError_t launch_batch_cholesky(int prec, const BatchDesc* desc, const int* order, const int* ld_rank,
                                 int count, double* factor, int* info, void* low, long factor_elems,
                                 hipStream_t st);

struct BatchSweepArgs {
  const BatchDesc* desc;
  const int* order;
  const double* L;         // factor base (FP64)
  const void* Llow;        // low-precision copy base (== L for FP64)
  const double* at;        // centred limits, packed like the inputs
  const double* bt;
  const uint64_t* lattice;
  uint64_t seed;
  int N, S, periodize, prec;
  void* yscr;
  long yslice;
  double* ell;             // count x N*S
  unsigned long long* counter;
  long total_items;        // count x chunks per problem
  long lplane;             // element distance of the BF16 hi and lo planes of the packed low copy
  int grid;
  int rows;                // rows per sweep block (128 or 64)
};

hipError_t launch_batch_setup(const BatchDesc* desc, int count, int nmax, const double* a, const double* b,
                              const double* mu, double* at, double* bt, int* bad,
                              unsigned long long* counter, hipStream_t st);
hipError_t launch_batch_sweep(const BatchSweepArgs& a, hipStream_t st);
// The sweeps with 256 sample columns per workgroup and four conditioning
// waves (kernels_sov_quad.hip): dense (SweepArgs with yslice = quad_yslice)
// and batched; 64-row blocks, or 128 for the reduced precisions.
hipError_t launch_quad_sweep(const SweepArgs& a, hipStream_t st);
hipError_t launch_quad_batch_sweep(const BatchSweepArgs& a, hipStream_t st);
int quad_sweep_cols();
// The FP64 sweep for few samples (kernels_sov_narrow.hip): 16 or 32 columns
// per three-wave workgroup, the next block's GEMM overlapped with the
// recurrence.
hipError_t launch_narrow_sweep(const SweepArgs& a, hipStream_t st);
int narrow_sweep_wg_per_cu(int cols);
int quad_wg_per_cu(int prec, int rows);
long quad_yslice(int prec, int ld);
hipError_t launch_batch_reduce(const double* ell, int count, int N, int S, double* part, const int* info,
                               const int* bad, double* out, hipStream_t st);

// ---------------------------------------------------------------- tile low rank
constexpr int kTlrMaxTile = 1024;   // largest TLR tile edge (LDS rows of the compression kernel)
constexpr int kTlrMaxRank = 256;    // largest rank cap (one lane per rank row in the row solves)
constexpr long kTlrPairBatch = 256; // tile pairs per update launch (sizes the WT / T workspace)
constexpr int kTlrRcGrid = 256;     // most recompression workgroups (one per CU, each with its scratch)
// Scratch doubles per recompression workgroup for tile edge m and rank
// stride rs: three rs x m and one m x rs blocks and seven rs x rs ones.
__host__ __device__ inline long tlr_rc_scratch_doubles(int m, int rs) { return 4L * rs * m + 7L * rs * rs; }

// Lower tiles of Sigma (tile-major, m x m each, identity past n) from the
// caller's Sigma or from locations with the Matern kernel; clears *info.
hipError_t launch_tlr_build(int n, int m, int nt, const double* sigma, int lds, const int64_t* perm,
                            const int* perm_bad, const double* locs, const Matern& mk, double* tiles, int* info,
                            hipStream_t st);

struct TlrCholArgs {
  double* tiles;     // nt(nt+1)/2 tiles of m x m
  double* U;         // nt(nt-1)/2 panels of m x rs
  double* Vt;        // nt(nt-1)/2 panels of rs x m (+ 128 rows of slack)
  int* ranks;        // nt(nt-1)/2
  int* info;         // global info (1 int)
  int* local_info;   // per-tile info scratch (1 int)
  double* WT;        // kTlrPairBatch x rs x rs
  double* T;         // kTlrPairBatch x m x rs
  double* rc_scratch;  // rc_grid x tlr_rc_scratch_doubles(m, rs) + a 64-byte counter, or nullptr: no recompression
  int rc_grid;
  int m, nt, rs, rcap;
  double eps;
};
hipError_t launch_tlr_cholesky(const TlrCholArgs& a, hipStream_t st);
// Recompression of every panel of a finished TLR factor to the smallest rank
// within eps (kernels_tlr.hip); grid workgroups with their scratch slots, the
// panel counter after them.
hipError_t launch_tlr_recompress(double* tiles, int m, int nt, int rs, double eps, double* U, double* Vt, int* ranks,
                                 double* scratch, int grid, const int* info, hipStream_t st);
// The TLR factor as a dense row-major lower factor D (ldd x ldd, ldd <= nt m):
// diagonal tiles copied, off-diagonal tiles U_ij V'^T_ij, zero / identity
// past n; the upper triangle is not written.
hipError_t launch_tlr_expand(int n, int m, int nt, int rs, const double* tiles, const double* U, const double* Vt,
                             const int* ranks, double* D, long ldd, hipStream_t st);

// Layout of the rank-dependent part of a TLR probability workspace,
// computed on the device from the factor's ranks (no read-back): byte
// offsets from the start of that part, and how many persistent sweep
// workgroups its size holds.
struct TlrSweepHdr {
  long ksum;     // stacked V' rows (sum of the ranks)
  long kpad;     // packed K of all tile-rows (Z rows)
  long vpack;    // (ksum + 128) x m doubles
  long upack;    // m x kpad doubles
  long yscr;     // grid x yslice doubles
  long zscr;     // grid x zslice doubles
  long zslice;   // kpad x 64
  long grid;     // workgroups that fit (0: not even one; the call's outputs are NaN)
};

// Index tables of the sweep (the layout of tlr_tables.h) and the header,
// from the ranks, by one workgroup.  dyn_bytes: size of the rank-dependent
// region; grid_max: the launch grid of the sweep; yslice: doubles of a
// workgroup's Y slice.  Sets *bad = 0 when no workgroup fits.
struct TlrTableArgs {
  const int* ranks;     // nt (nt - 1) / 2
  int nt, rs, m;
  int ext_pack;         // the packed operands live in the factor (compact): no room for them in dyn
  long yslice;
  long grid_max;
  size_t dyn_bytes;
  int cols;             // sample columns per sweep workgroup (Z slice kpad x cols): 64, or 256 (four-wave sweep)
  int* kk;              // per pair: rank used (|rank| clipped to rs)
  long* zcol;           // nt + 1
  long* kpad0;          // nt + 1
  int* kval;            // nt
  long* vrow0;          // per pair
  long* ucol0;          // per pair
  long* zdst;           // np * rs (the first ksum entries are used)
  TlrSweepHdr* hdr;
  int* bad;
};
hipError_t launch_tlr_tables(const TlrTableArgs& a, hipStream_t st);

// Packing of the low-rank factors for the sweep (into the rank-dependent
// region `dyn` at the header's offsets).
struct TlrPackArgs {
  const double* U;      // factor: per pair m x rs
  const double* Vt;     // factor: per pair rs x m
  int m, rs, np;
  const int* kk;        // per pair: rank used
  const long* vrow0;    // per pair: first stacked V' row
  const long* ucol0;    // per pair: first packed column within its tile-row
  const long* kpad0;    // nt + 1
  const int* kval;      // nt
  const TlrSweepHdr* hdr;
  char* dyn;
};
hipError_t launch_tlr_pack(const TlrPackArgs& a, hipStream_t st);

struct TlrSweepArgs {
  const double* tiles;  // factor tiles (the dense diagonal tiles are read)
  const TlrSweepHdr* hdr;  // Vpack, Upack, Y and Z scratch at its offsets from dyn
  char* dyn;
  const long* zcol;     // nt + 1: first stacked V' row of tile column j
  const long* kpad0;    // nt + 1: first packed K index (Z row) of tile-row i
  const int* kval;      // nt: K_i, rows [K_i, Kpad_i) of tile-row i are padding
  const long* zdst;     // ksum: Z row of stacked V' row
  int m, nt, n;
  const double* at;
  const double* bt;
  const uint64_t* lattice;
  uint64_t seed;
  int N, S, periodize;
  long yslice;      // (nt m) x 64, or (nt m) x 256 for the four-wave sweep
  double* ell;
  int grid;         // launch grid (workgroups past hdr->grid leave at once)
  int rows;         // rows per sweep block: 128 (two workgroups per CU) or 64 (four); 256 selects the
                    // four-wave sweep (256 columns per workgroup, 64-row blocks; yslice (nt m) x 256)
  double* prefix;   // nullptr, or n x nchunks x 4 partials of the running products per row
  const double* vpack_ext;  // compact factor: its packed V' rows and U columns (else nullptr:
  const double* upack_ext;  //   the copies in dyn at the header's offsets)
  int diag_compact;         // diagonal tile i at i m^2 (compact) instead of (i(i+1)/2 + i) m^2
};
hipError_t launch_tlr_sweep(const TlrSweepArgs& a, hipStream_t st);
// The four-wave form (kernels_sov_quad.hip), launched by launch_tlr_sweep for rows == 256.
hipError_t launch_quad_tlr_sweep(const TlrSweepArgs& a, hipStream_t st);

}  // namespace mvn
