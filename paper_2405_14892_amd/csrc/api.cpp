// C ABI of the library (declared in include/mvn.h): argument validation,
// workspace carving, the Richtmyer lattice table, and the launch sequences.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/mvn.h"
#include "launch.h"
#include "tlr_tables.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e));
  return -1000 - (int)e;
}

constexpr size_t kAlign = 256;
constexpr int kCUs = 256;      // compute units of an MI355X: the persistent grids are sized for it
// Automatic narrow sweep: at most kNarrowMaxNS samples, and samples x
// dimensions at most kNarrowMaxWork16 with 16-column chunks (up to 12 288
// samples), kNarrowMaxWork32 with 32-column ones.  Measured (FP64, one box,
// 64-column sweep against the narrow one, 10^4 samples): 4096 sites 11.9 /
// 9.2 ms, 6144 sites 20.0 / 18.5 ms, 8192 sites 31.9 / 31.0 ms, 12 288 sites
// 63.6 / 69.9 ms; 4096 sites with 2 x 10^4 samples (32 columns) 15.2 / 17.7
// ms.  Each narrow workgroup streams the whole factor, so the factor's size
// bounds it.
constexpr long kNarrowMaxNS = 20480;
constexpr double kNarrowMaxWork16 = 9e7, kNarrowMaxWork32 = 4.5e7;

// Rows per sweep block: 0 selects the default (128); 32 (the narrow FP64
// sweep of dense factors) runs its own 32-row blocks, and the other sweeps
// take 128 then.
int sweep_rows(const mvn_options* o) {
  return (!o || o->sweep_rows == 0 || o->sweep_rows == 32) ? 128 : o->sweep_rows;
}
// The raw option (0 = automatic choice of the dense sweep).
int rows_opt(const mvn_options* o) { return o ? o->sweep_rows : 0; }
// The TLR sweep's blocks: its GEMMs are short (packed ranks plus the dense
// part of one tile), so conditioning dominates and 64-row blocks (four
// workgroups per CU) are the default.
// TLR sweeps: 64- or 128-row blocks of 64 columns per workgroup (0 = 64), or
// 256: the four-wave sweep, 256 columns per workgroup and 64-row blocks, on
// request only (at 65 536 sites it beat the 64-row blocks by 2% at N*S = 10^5
// and lost at 32 768, 65 536, 131 072 and 200 000 samples).
int tlr_sweep_rows(const mvn_options* o, long) {
  if (!o || o->sweep_rows == 0) return 64;
  return o->sweep_rows;
}
bool tlr_rows_ok(const mvn_options* o) {
  return !o || o->sweep_rows == 0 || o->sweep_rows == 64 || o->sweep_rows == 128 || o->sweep_rows == 256;
}
bool sweep_rows_ok(const mvn_options* o) { return !o || o->sweep_rows == 0 || o->sweep_rows == 64 || o->sweep_rows == 128; }
// Dense probability and nested-set sweeps also take 32 (FP64 only).
bool dense_rows_ok(const mvn_options* o) {
  return sweep_rows_ok(o) || (o->sweep_rows == 32 && o->precision == MVN_FP64);
}
int max_grid(int rows, int prec) { return kCUs * mvn::sweep_wg_per_cu(rows, prec); }

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int padded(int n) { return (n + 127) / 128 * 128; }

// Kernel parameters for the build kernels (unused when Sigma is given).
mvn::Matern matern_of(const mvn_matern* k) {
  return k ? mvn::make_matern(k->sigma2, k->beta, k->nu, k->nugget) : mvn::make_matern(1.0, 1.0, 0.5, 0.0);
}

// Header of a dense factor buffer, after L: info (int), max diag(Sigma) at
// +8, the adaptive map's three update counters at +16, and two slots of
// ld/128 + 1 panel block norms at +64.
size_t dense_header_bytes(int ld) { return align_up(64 + sizeof(double) * 2 * ((size_t)ld / 128 + 1)); }

int elem_bytes_low(int prec) { return prec == MVN_FP32 ? 4 : prec == MVN_BF16 ? 2 : prec == MVN_BF16X3 ? 4 : 0; }
bool prec_ok(int prec) { return prec >= MVN_FP64 && prec <= MVN_BF16X3; }

bool opts_ok(const mvn_options* o, int* arg_bad_tile) {
  if (!o) return true;
  *arg_bad_tile = 0;
  if (o->tile < 16 || o->tile % 4 != 0) *arg_bad_tile = 1;
  return *arg_bad_tile == 0;
}

// ---------------------------------------------------------------- lattice
// A_i = floor(frac(sqrt(p_{i+1})) 2^64) with exact integer arithmetic:
// q = floor(sqrt p), r = p - q^2, F is the largest integer with
// (q 2^64 + F)^2 <= p 2^128, i.e. F^2 + 2 q F 2^64 <= r 2^128.
bool frac_ok(uint64_t q, uint64_t r, uint64_t F) {
  const unsigned __int128 sq = (unsigned __int128)F * F;
  const unsigned __int128 hi = sq >> 64;
  const uint64_t lo = (uint64_t)sq;
  const unsigned __int128 lhs = hi + (unsigned __int128)2 * q * F;
  const unsigned __int128 rhs = (unsigned __int128)r << 64;
  return lhs < rhs || (lhs == rhs && lo == 0);
}

uint64_t frac_sqrt_2p64(uint64_t p) {
  uint64_t q = (uint64_t)sqrtl((long double)p);
  while (q * q > p) --q;
  while ((q + 1) * (q + 1) <= p) ++q;
  const uint64_t r = p - q * q;
  long double est = ldexpl((long double)r / (sqrtl((long double)p) + (long double)q), 64);
  uint64_t F = est >= 18446744073709551615.0L ? UINT64_MAX : (uint64_t)est;
  while (!frac_ok(q, r, F)) --F;
  while (F != UINT64_MAX && frac_ok(q, r, F + 1)) ++F;
  return F;
}

std::mutex g_lat_mu;
uint64_t* g_lat_host = nullptr;   // pinned; grow-only (older tables stay alive)
int g_lat_n = 0;

const uint64_t* lattice_table(int n) {
  std::lock_guard<std::mutex> lk(g_lat_mu);
  if (n <= g_lat_n) return g_lat_host;
  // the first table already covers 131072 dimensions, so that later calls
  // (possibly under graph capture) up to that size allocate nothing
  int want = n < (1 << 17) ? (1 << 17) : n;
  // sieve enough primes: p_k < k (ln k + ln ln k) for k >= 6
  const double lw = log((double)want + 16);
  size_t limit = (size_t)(want * (lw + log(lw) + 3)) + 64;
  std::vector<uint8_t> comp(limit + 1, 0);
  std::vector<uint64_t> primes;
  primes.reserve(want);
  for (size_t v = 2; v <= limit && (int)primes.size() < want; ++v) {
    if (comp[v]) continue;
    primes.push_back(v);
    for (size_t m = v * v; m <= limit; m += v) comp[m] = 1;
  }
  if ((int)primes.size() < want) return nullptr;
  uint64_t* buf = nullptr;
  if (hipHostMalloc((void**)&buf, sizeof(uint64_t) * want, hipHostMallocDefault) != hipSuccess)
    return nullptr;
  for (int i = 0; i < want; ++i) buf[i] = frac_sqrt_2p64(primes[i]);
  g_lat_host = buf;  // the previous table is deliberately kept: in-flight copies may read it
  g_lat_n = want;
  return buf;
}

struct ProbLayout {
  size_t at, bt, lat, ell, part, bad, yscr, zscr, total;
  int ld, grid;
  long yslice, zslice;
};

// Which dense sweep kernel runs a call.
enum SweepKind { kSweep64 = 0, kSweepWide = 1, kSweepQuad = 2, kSweepNarrow = 3 };

// Columns per workgroup of the narrow sweep: 16 while the chunks fit its
// workgroup slots, else 32.
int narrow_cols(long NS) { return (NS + 15) / 16 <= (long)kCUs * mvn::narrow_sweep_wg_per_cu(16) ? 16 : 32; }

// Workspace of one probability call.  ld is the factor's leading dimension
// (rows of the Y scratch); zslice > 0 adds the TLR Z scratch (FP64).
// kSweepWide: the 128-column FP64 sweep (persistent workgroups, each owning
// whole 32-column slices; Y slice ld x 128); kSweepQuad: 256 columns per
// workgroup, four conditioning waves.
ProbLayout prob_layout_ld(int ld, int N, int S, int prec, long zslice, int rows, int kind = kSweep64,
                          int gcap = 0) {
  ProbLayout L{};
  L.ld = ld;
  const long NS = (long)N * S;
  if (kind == kSweepNarrow) {
    const int cols = narrow_cols(NS);
    const long chunks = (NS + cols - 1) / cols;
    const int gmax = mvn::narrow_sweep_wg_per_cu(cols) * kCUs;
    L.grid = (int)(chunks < gmax ? chunks : gmax);
    L.yslice = (long)L.ld * cols;
  } else if (kind == kSweepWide) {
    const long slices = (NS + 31) / 32;
    const int gmax = mvn::wide_sweep_wg_per_cu() * kCUs;
    L.grid = (int)(slices < gmax ? slices : gmax);
    L.yslice = (long)L.ld * mvn::wide_sweep_cols();
  } else if (kind == kSweepQuad) {
    const long chunks = (NS + mvn::quad_sweep_cols() - 1) / mvn::quad_sweep_cols();
    const int gmax = mvn::quad_wg_per_cu(prec, rows) * kCUs;
    L.grid = (int)(chunks < gmax ? chunks : gmax);
    L.yslice = mvn::quad_yslice(prec, L.ld);
  } else {
    const long chunks = (NS + mvn::sweep_tile_cols() - 1) / mvn::sweep_tile_cols();
    const int gmax = max_grid(rows, prec);
    L.grid = (int)(chunks < gmax ? chunks : gmax);
    L.yslice = mvn::sweep_yslice(prec, L.ld);
  }
  if (gcap > 0 && L.grid > gcap) L.grid = gcap;
  L.zslice = zslice;
  size_t off = 0;
  L.at = off; off = align_up(off + sizeof(double) * L.ld);
  L.bt = off; off = align_up(off + sizeof(double) * L.ld);
  L.lat = off; off = align_up(off + sizeof(uint64_t) * L.ld);
  L.ell = off; off = align_up(off + sizeof(double) * (size_t)NS);
  L.part = off; off = align_up(off + sizeof(double) * 2 * (size_t)S);
  L.bad = off; off = align_up(off + sizeof(int));
  L.yscr = off;
  off = align_up(off + (size_t)mvn::sweep_elem_bytes(prec) * (size_t)L.grid * L.yslice);
  L.zscr = off;
  off = align_up(off + sizeof(double) * (size_t)L.grid * (size_t)zslice);
  L.total = off;
  return L;
}

// The dense sweep's workspace; `prefix`: for a nested-set sweep (which keeps
// the 64-column kernel).
// The 128-column sweep needs enough samples for full passes (a workgroup
// per 128 columns on every CU slot); with fewer, the 64-column sweep reads
// the factor no more often and runs more workgroups.
bool use_wide(int prec, int rows, bool prefix, long NS) {
  return prec == MVN_FP64 && rows == 128 && !prefix &&
         NS >= (long)mvn::wide_sweep_wg_per_cu() * kCUs * mvn::wide_sweep_cols();
}

// Reduced-precision operands with 128-row blocks run the four-wave sweep
// when its 256-column chunks fill every workgroup slot (measured on the
// 16384-site problem: BF16 282 against 456 ms, split BF16 976 against 1065,
// FP32 579 against 604; the FP64 and few-sample sweeps are faster with 64
// columns per workgroup).
// The narrow sweep (FP64; sweep_rows 32, or 0 with few samples and sites):
// with few samples the 64-column sweep leaves CUs idle and each workgroup's
// time is its own chain of n steps plus its GEMM.
// rows_raw: the sweep_rows option as given (0 = automatic).
int sweep_kind(int prec, int rows_raw, bool prefix, long NS, int n) {
  if (prec == MVN_FP64 &&
      (rows_raw == 32 || (rows_raw == 0 && NS <= kNarrowMaxNS &&
                          (double)NS * n <= (narrow_cols(NS) == 16 ? kNarrowMaxWork16 : kNarrowMaxWork32))))
    return kSweepNarrow;
  const int rows = rows_raw == 0 || rows_raw == 32 ? 128 : rows_raw;
  if (use_wide(prec, rows, prefix, NS)) return kSweepWide;
  const long chunks = (NS + mvn::quad_sweep_cols() - 1) / mvn::quad_sweep_cols();
  if (prec != MVN_FP64 && rows == 128 && chunks >= (long)kCUs * mvn::quad_wg_per_cu(prec, rows)) return kSweepQuad;
  return kSweep64;
}

ProbLayout prob_layout(int n, int N, int S, int prec, int rows_raw, bool prefix = false) {
  const int rows = rows_raw == 0 || rows_raw == 32 ? 128 : rows_raw;
  return prob_layout_ld(padded(n), N, S, prec, 0, rows, sweep_kind(prec, rows_raw, prefix, (long)N * S, n));
}

// Sample columns per chunk of a dense sweep's nested-set partials.
int prefix_cols(int prec, int rows_raw, long NS, int n) {
  return sweep_kind(prec, rows_raw, true, NS, n) == kSweepNarrow ? narrow_cols(NS) : mvn::sweep_tile_cols();
}

// Front of the workspace of a nested-set call: the running-product partials
// of the prefix sweep (n x nchunks x 4 doubles) and the per-shift estimates
// of every prefix (n x S doubles); the probability workspace follows.
struct PrefixRegion {
  size_t part, lps, total;
  long nchunks;
  int cols;
};

PrefixRegion prefix_region(int n, int N, int S, int cols) {
  PrefixRegion P{};
  P.cols = cols;
  P.nchunks = ((long)N * S + cols - 1) / cols;
  size_t off = 0;
  P.part = off; off = align_up(off + sizeof(double) * 4 * (size_t)n * (size_t)P.nchunks);
  P.lps = off; off = align_up(off + sizeof(double) * (size_t)n * (size_t)S);
  P.total = off;
  return P;
}

// Workspace of a Monte Carlo check: first-failure bins, the work counter and
// the per-workgroup Z scratch.
struct McLayout {
  size_t hist, counter, yscr, total;
  int grid, rows;
  long yslice;
};

int mc_rows(const mvn_options* o) { return (!o || o->sweep_rows == 0) ? 128 : o->sweep_rows; }

McLayout mc_layout(int n, long M, int rows) {
  McLayout L{};
  L.rows = rows;
  const long chunks = (M + mvn::sweep_tile_cols() - 1) / mvn::sweep_tile_cols();
  const long gmax = (long)kCUs * mvn::mc_wg_per_cu(rows);
  L.grid = (int)(chunks < gmax ? chunks : gmax);
  L.yslice = (long)padded(n) * mvn::sweep_tile_cols();
  size_t off = 0;
  L.hist = off; off = align_up(off + sizeof(unsigned long long) * ((size_t)n + 1));
  L.counter = off; off = align_up(off + sizeof(unsigned long long));
  L.yscr = off; off = align_up(off + sizeof(double) * (size_t)L.grid * (size_t)L.yslice);
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- tile low rank
// Factor buffer of a TLR factor: tiles | info | U | Vt (+128 rows) | ranks.
struct TlrGeom {
  int m, nt, rs, ld;
  long ntiles, npanels;
  size_t tiles, info, U, Vt, ranks, total;
  size_t ws_local, ws_wt, ws_t, ws_rc, ws_total;  // factorisation workspace
  int rc_grid;
};

TlrGeom tlr_geom(int n, int m, int max_rank) {
  TlrGeom G{};
  G.m = m;
  G.nt = (n + m - 1) / m;
  G.ld = G.nt * m;
  G.rs = (max_rank + 15) / 16 * 16;
  G.ntiles = (long)G.nt * (G.nt + 1) / 2;
  G.npanels = (long)G.nt * (G.nt - 1) / 2;
  size_t off = 0;
  G.tiles = off; off = align_up(off + sizeof(double) * (size_t)G.ntiles * m * m);
  G.info = off; off = align_up(off + sizeof(int));
  G.U = off; off = align_up(off + sizeof(double) * (size_t)G.npanels * m * G.rs);
  G.Vt = off; off = align_up(off + sizeof(double) * ((size_t)G.npanels * G.rs + 128) * m);
  G.ranks = off; off = align_up(off + sizeof(int) * (size_t)(G.npanels > 0 ? G.npanels : 1));
  G.total = off;
  const long batch = std::min<long>(mvn::kTlrPairBatch, G.npanels > 0 ? G.npanels : 1);
  size_t w = 0;
  G.ws_local = w; w = align_up(w + sizeof(int));
  G.ws_wt = w; w = align_up(w + sizeof(double) * (size_t)batch * G.rs * G.rs);
  G.ws_t = w; w = align_up(w + sizeof(double) * (size_t)batch * m * G.rs);
  // recompression: one workgroup per panel, at most kTlrRcGrid
  G.rc_grid = (int)std::min<long>(mvn::kTlrRcGrid, G.npanels);
  // (+ the panel counter after the slots)
  G.ws_rc = w;
  w = align_up(w + sizeof(double) * (size_t)G.rc_grid * (size_t)mvn::tlr_rc_scratch_doubles(m, G.rs) + 64);
  G.ws_total = w;
  return G;
}

// 0 if the TLR options are usable, else writes the message and returns 1.
int tlr_opts_check(const mvn_options* o) {
  if (o->precision != MVN_FP64) return fail(1, "tile low-rank factors are FP64 (precision %d)", o->precision);
  if (o->tile < 128 || o->tile > mvn::kTlrMaxTile || o->tile % 128 != 0)
    return fail(1, "TLR tile must be a multiple of 128 in [128, %d] (got %d)", mvn::kTlrMaxTile, o->tile);
  if (o->max_rank < 1 || o->max_rank > mvn::kTlrMaxRank || o->max_rank > o->tile)
    return fail(1, "TLR max_rank must be in [1, min(%d, tile)] (got %d)", mvn::kTlrMaxRank, o->max_rank);
  return 0;
}

bool is_tlr(const mvn_options* o) { return o && o->tlr_eps > 0; }

// Workspace of a TLR probability call: the common part of prob_layout_ld (up
// to the invalid-limit flag), the sweep's index tables (tlr_tables.h, built
// on the device from the ranks) and the device header of the rank-dependent
// region, then that region: the packed operands, and per persistent
// workgroup its Y slice (ld x 64) and Z slice (kpad x 64).  The fixed part
// depends only on the factor's geometry (zdst is sized for every tile at
// the rank stride); the region's layout is computed on the device
// (TlrSweepHdr), and `dyn_bytes(ksum, kpad, grid)` gives the size it needs
// for given ranks and workgroups, the same arithmetic as the device's.
struct TlrProbLayout {
  ProbLayout base;
  size_t kk, zcol, kpad0, kval, vrow0, ucol0, zdst, hdr, fixed;
  long yslice;
  int cols;       // sample columns per workgroup: 64, or 256 (four-wave sweep)
  int grid;       // launch grid (the device runs as many as the region holds)
  bool ext_pack;  // compact factor: the packed operands are the factor's, not in the region
  size_t dyn_bytes(long ksum, long kpad, long g, int m) const {
    const size_t kp = kpad > 0 ? (size_t)kpad : 1;
    const size_t ysc = ext_pack ? 0 : align_up(8 * (size_t)(ksum + 128) * m) + align_up(8 * (size_t)m * kp);
    return ysc + (size_t)g * (align_up(8 * (size_t)yslice) + align_up(8 * kp * (size_t)cols));
  }
};

bool is_compact(const mvn_factor* f) { return (f->flags & MVN_FACTOR_TLR_COMPACT) != 0; }

TlrProbLayout tlr_prob_layout(int ld, int nt, int rs, int N, int S, int rows, bool ext_pack = false) {
  TlrProbLayout L{};
  L.ext_pack = ext_pack;
  const bool quad = rows == 256;
  L.base = quad ? prob_layout_ld(ld, N, S, MVN_FP64, 0, 64, kSweepQuad) : prob_layout_ld(ld, N, S, MVN_FP64, 0, rows);
  const size_t np = (size_t)nt * (nt - 1) / 2;
  const size_t np1 = np > 0 ? np : 1;
  size_t off = L.base.yscr;
  L.kk = off; off = align_up(off + sizeof(int) * np1);
  L.zcol = off; off = align_up(off + sizeof(long) * (nt + 1));
  L.kpad0 = off; off = align_up(off + sizeof(long) * (nt + 1));
  L.kval = off; off = align_up(off + sizeof(int) * nt);
  L.vrow0 = off; off = align_up(off + sizeof(long) * np1);
  L.ucol0 = off; off = align_up(off + sizeof(long) * np1);
  L.zdst = off; off = align_up(off + sizeof(long) * np1 * rs);
  L.hdr = off; off = align_up(off + sizeof(mvn::TlrSweepHdr));
  L.fixed = off;
  L.cols = quad ? mvn::quad_sweep_cols() : mvn::sweep_tile_cols();
  L.yslice = (long)ld * L.cols;
  L.grid = L.base.grid;
  return L;
}

// Ranks of a TLR factor, read back with a synchronisation of `stream`.
hipError_t tlr_read_ranks(const mvn_factor* f, std::vector<int>& r, hipStream_t stream) {
  const int nt = f->ld / f->tile;
  const long np = (long)nt * (nt - 1) / 2;
  r.assign(np > 0 ? np : 1, 0);
  if (np == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(r.data(), f->ranks, sizeof(int) * np, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(stream);
}

struct GradLayout {
  size_t at, bt, lat, ell, part, bad, yscr, sfw, sbar, gpart, mz, scale, total;
  int ld, grid;
  long nchunks;
};

GradLayout grad_layout(int n, int N, int S) {
  GradLayout L{};
  L.ld = padded(n);
  const long NS = (long)N * S;
  L.nchunks = (NS + mvn::sweep_tile_cols() - 1) / mvn::sweep_tile_cols();
  L.grid = (int)(L.nchunks < max_grid(128, 0) ? L.nchunks : max_grid(128, 0));
  const size_t slice = sizeof(double) * (size_t)L.ld * mvn::sweep_tile_cols();
  size_t off = 0;
  L.at = off; off = align_up(off + sizeof(double) * L.ld);
  L.bt = off; off = align_up(off + sizeof(double) * L.ld);
  L.lat = off; off = align_up(off + sizeof(uint64_t) * L.ld);
  L.ell = off; off = align_up(off + sizeof(double) * (size_t)NS);
  L.part = off; off = align_up(off + sizeof(double) * 2 * (size_t)S);
  L.bad = off; off = align_up(off + sizeof(int));
  L.yscr = off; off = align_up(off + slice * L.grid);
  L.sfw = off; off = align_up(off + slice * L.grid);
  L.sbar = off; off = align_up(off + slice * L.grid);
  L.gpart = off; off = align_up(off + sizeof(double) * 2 * (size_t)L.ld * L.nchunks);
  L.mz = off; off = align_up(off + sizeof(double) * 2 * (size_t)L.nchunks);
  L.scale = off; off = align_up(off + sizeof(double) * ((size_t)L.nchunks + 1));
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- batches
struct BatchPlan {
  std::vector<mvn::BatchDesc> desc;
  std::vector<int> order, ld_rank;
  long factor_elems = 0, total_tiles = 0, sum_n = 0;
  int nmax = 0, ldmax = 0;
};

bool batch_plan_host(int count, const int* n_p, BatchPlan& P) {
  P.desc.resize(count);
  P.order.resize(count);
  long fo = 0, lo = 0, to = 0;
  for (int p = 0; p < count; ++p) {
    if (n_p[p] < 1) return false;
    mvn::BatchDesc& d = P.desc[p];
    d.n = n_p[p];
    d.ld = padded(n_p[p]);
    d.factor_off = fo;
    d.lim_off = lo;
    d.tile_off = to;
    d.reserved = 0;
    fo += (long)d.ld * d.ld;
    lo += d.n;
    const long nb = d.ld / 64;
    to += nb * (nb + 1) / 2;
    P.nmax = d.n > P.nmax ? d.n : P.nmax;
  }
  P.factor_elems = fo;
  P.sum_n = lo;
  P.total_tiles = to;
  for (int p = 0; p < count; ++p) P.order[p] = p;
  std::stable_sort(P.order.begin(), P.order.end(), [&](int x, int y) { return n_p[x] > n_p[y]; });
  P.ld_rank.resize(count);
  for (int r = 0; r < count; ++r) P.ld_rank[r] = P.desc[P.order[r]].ld;
  P.ldmax = P.ld_rank[0];
  return true;
}

size_t batch_plan_bytes(int count) {
  return align_up(sizeof(mvn::BatchDesc) * (size_t)count) + align_up(sizeof(int) * (size_t)count);
}

size_t batch_factor_bytes(const BatchPlan& P, int prec) {
  return align_up(sizeof(double) * (size_t)P.factor_elems) + align_up((size_t)elem_bytes_low(prec) * P.factor_elems);
}

struct BatchWs {
  size_t at, bt, lat, ell, part, bad, counter, yscr, total;
  int grid;
  long items, yslice;
};

// The batch sweep with four conditioning waves per workgroup (256 columns
// per work item), except FP64 with 128-row blocks (the 64-column sweep).
bool batch_quad(int prec, int rows) { return rows == 64 || prec != MVN_FP64; }

BatchWs batch_ws(const BatchPlan& P, int count, int N, int S, int prec, int rows) {
  BatchWs W{};
  const long NS = (long)N * S;
  const bool quad = batch_quad(prec, rows);
  const int cols = quad ? mvn::quad_sweep_cols() : mvn::sweep_tile_cols();
  const long chunks = (NS + cols - 1) / cols;
  W.items = chunks * count;
  const int gmax = quad ? kCUs * mvn::quad_wg_per_cu(prec, rows) : max_grid(rows, prec);
  W.grid = (int)(W.items < gmax ? W.items : gmax);
  W.yslice = quad ? mvn::quad_yslice(prec, P.ldmax) : mvn::sweep_yslice(prec, P.ldmax);
  size_t off = 0;
  W.at = off; off = align_up(off + sizeof(double) * (size_t)P.sum_n);
  W.bt = off; off = align_up(off + sizeof(double) * (size_t)P.sum_n);
  W.lat = off; off = align_up(off + sizeof(uint64_t) * (size_t)P.ldmax);
  W.ell = off; off = align_up(off + sizeof(double) * (size_t)NS * count);
  W.part = off; off = align_up(off + sizeof(double) * 2 * (size_t)S * count);
  W.bad = off; off = align_up(off + sizeof(int) * (size_t)count);
  W.counter = off; off = align_up(off + sizeof(unsigned long long));
  W.yscr = off;
  off = align_up(off + (size_t)mvn::sweep_elem_bytes(prec) * (size_t)W.grid * W.yslice);
  W.total = off;
  return W;
}

// The dense sweep and reduction of mvn_prob into a validated workspace; with
// prefix (the partials of a nested-set call) the sweep also records the
// running products of every row and no full reduction is launched.
// dlat_dev: a lattice table already on the device (at least n entries), or
// nullptr to copy the host table into the workspace.
int dense_sweep(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int N, int S,
                uint64_t seed, const mvn_options* opts, void* ws, const ProbLayout& Lay, double* d_ell,
                double* prefix, double* d_out, hipStream_t stream, const uint64_t* dlat_dev = nullptr) {
  const int n = f->n;
  const int prec = opts->precision;
  const int rows = sweep_rows(opts);
  char* w = (char*)ws;
  double* at = (double*)(w + Lay.at);
  double* bt = (double*)(w + Lay.bt);
  const uint64_t* dlat = dlat_dev;
  double* ell = d_ell ? d_ell : (double*)(w + Lay.ell);
  double* part = (double*)(w + Lay.part);
  int* bad = (int*)(w + Lay.bad);
  void* yscr = (void*)(w + Lay.yscr);
  hipError_t e;
  if (!dlat) {
    const uint64_t* lat = lattice_table(n);
    if (!lat) return fail(-1, "could not build the lattice table for n = %d", n);
    uint64_t* dl = (uint64_t*)(w + Lay.lat);
    e = hipMemcpyAsync(dl, lat, sizeof(uint64_t) * n, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "lattice copy");
    dlat = dl;
  }
  e = mvn::launch_prob_setup(n, f->ld, d_a, d_b, d_mu, at, bt, bad, stream);
  if (e != hipSuccess) return hip_fail(e, "setup");
  mvn::SweepArgs sa{};
  sa.L = f->L;
  sa.Llow = prec == MVN_FP64 ? (const void*)f->L : f->L_low;
  sa.prec = prec;
  sa.yslice = Lay.yslice;
  sa.ld = f->ld;
  sa.n = n;
  sa.at = at;
  sa.bt = bt;
  sa.lattice = dlat;
  sa.seed = seed;
  sa.N = N;
  sa.S = S;
  sa.periodize = opts->periodize ? 1 : 0;
  sa.yscr = yscr;
  sa.ell = ell;
  sa.grid = Lay.grid;
  sa.rows = rows;
  sa.prefix = prefix;
  const int kind = sweep_kind(prec, rows_opt(opts), prefix != nullptr, (long)N * S, n);
  sa.wide = kind == kSweepWide ? 1 : 0;
  sa.quad = kind == kSweepQuad ? 1 : 0;
  sa.narrow = kind == kSweepNarrow ? narrow_cols((long)N * S) : 0;
  e = mvn::launch_sweep(sa, stream);
  if (e != hipSuccess) return hip_fail(e, "sweep");
  if (prefix) return 0;
  e = mvn::launch_reduce(ell, N, S, part, f->info, bad, d_out, stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  return 0;
}

// The TLR sweep and reduction of mvn_prob (options validated by the
// caller): the index tables and the layout of the rank-dependent region are
// built on the device from the factor's ranks (nothing is read back and the
// stream is not synchronised), the low-rank factors are packed, the sweep
// runs as many persistent workgroups as the workspace holds, and the
// reduction follows.  With prefix (the partials of a nested-set call) the
// sweep also records the running products of every row, no full reduction
// is launched, and *bad_out gets the invalid-limit flag.
int tlr_sweep_call(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int N, int S,
                   uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes, double* d_ell,
                   double* prefix, double* d_out, hipStream_t stream, const int** bad_out) {
  const int rows = tlr_sweep_rows(opts, (long)N * S);
  const int n = f->n, m = f->tile, nt = f->ld / f->tile, rs = f->rank_stride;
  const int np = nt * (nt - 1) / 2;
  const bool compact = is_compact(f);
  const TlrProbLayout Lay = tlr_prob_layout(f->ld, nt, rs, N, S, rows, compact);
  const size_t least = Lay.fixed + Lay.dyn_bytes(0, 0, 1, m);
  if (ws_bytes < least)
    return fail(-10, "workspace too small: %zu bytes hold no sweep workgroup (at least %zu)", ws_bytes, least);
  const uint64_t* lat = lattice_table(n);
  if (!lat) return fail(-1, "could not build the lattice table for n = %d", n);
  char* w = (char*)ws;
  double* at = (double*)(w + Lay.base.at);
  double* bt = (double*)(w + Lay.base.bt);
  uint64_t* dlat = (uint64_t*)(w + Lay.base.lat);
  double* ell = d_ell ? d_ell : (double*)(w + Lay.base.ell);
  double* part = (double*)(w + Lay.base.part);
  int* bad = (int*)(w + Lay.base.bad);
  mvn::TlrSweepHdr* hdr = (mvn::TlrSweepHdr*)(w + Lay.hdr);
  char* dyn = w + Lay.fixed;
  hipError_t e = hipMemcpyAsync(dlat, lat, sizeof(uint64_t) * n, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "lattice copy");
  e = mvn::launch_prob_setup(n, f->ld, d_a, d_b, d_mu, at, bt, bad, stream);
  if (e != hipSuccess) return hip_fail(e, "setup");
  mvn::TlrTableArgs tb{};
  tb.ranks = f->ranks;
  tb.nt = nt;
  tb.rs = rs;
  tb.m = m;
  tb.ext_pack = compact ? 1 : 0;
  tb.yslice = Lay.yslice;
  tb.cols = Lay.cols;
  tb.grid_max = Lay.grid;
  tb.dyn_bytes = ws_bytes - Lay.fixed;
  tb.kk = (int*)(w + Lay.kk);
  tb.zcol = (long*)(w + Lay.zcol);
  tb.kpad0 = (long*)(w + Lay.kpad0);
  tb.kval = (int*)(w + Lay.kval);
  tb.vrow0 = (long*)(w + Lay.vrow0);
  tb.ucol0 = (long*)(w + Lay.ucol0);
  tb.zdst = (long*)(w + Lay.zdst);
  tb.hdr = hdr;
  tb.bad = bad;
  e = mvn::launch_tlr_tables(tb, stream);
  if (e != hipSuccess) return hip_fail(e, "tlr tables");
  mvn::TlrPackArgs pa{};
  pa.U = f->U;
  pa.Vt = f->Vt;
  pa.m = m;
  pa.rs = rs;
  pa.np = np;
  pa.kk = tb.kk;
  pa.vrow0 = tb.vrow0;
  pa.ucol0 = tb.ucol0;
  pa.kpad0 = tb.kpad0;
  pa.kval = tb.kval;
  pa.hdr = hdr;
  pa.dyn = dyn;
  if (!compact) {
    e = mvn::launch_tlr_pack(pa, stream);
    if (e != hipSuccess) return hip_fail(e, "tlr pack");
  }
  mvn::TlrSweepArgs ta{};
  ta.tiles = f->L;
  ta.hdr = hdr;
  ta.dyn = dyn;
  ta.zcol = tb.zcol;
  ta.kpad0 = tb.kpad0;
  ta.kval = tb.kval;
  ta.zdst = tb.zdst;
  ta.m = m;
  ta.nt = nt;
  ta.n = n;
  ta.at = at;
  ta.bt = bt;
  ta.lattice = dlat;
  ta.seed = seed;
  ta.N = N;
  ta.S = S;
  ta.periodize = opts->periodize ? 1 : 0;
  ta.yslice = Lay.yslice;
  ta.ell = ell;
  ta.grid = Lay.grid;
  ta.rows = rows;
  ta.prefix = prefix;
  ta.vpack_ext = compact ? f->Vt : nullptr;
  ta.upack_ext = compact ? f->U : nullptr;
  ta.diag_compact = compact ? 1 : 0;
  e = mvn::launch_tlr_sweep(ta, stream);
  if (e != hipSuccess) return hip_fail(e, "tlr sweep");
  if (prefix) {
    *bad_out = bad;
    return 0;
  }
  e = mvn::launch_reduce(ell, N, S, part, f->info, bad, d_out, stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  return 0;
}

}  // namespace

extern "C" {

const char* mvn_last_error(void) { return g_err; }

int mvn_version(void) { return 100; }

int mvn_factor_bytes(int n, const mvn_options* opts, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (!bytes) return fail(-3, "bytes is NULL");
  const int prec = opts ? opts->precision : MVN_FP64;
  if (!prec_ok(prec)) return fail(-2, "unknown precision %d", prec);
  if (is_tlr(opts)) {
    if (tlr_opts_check(opts)) return -2;
    *bytes = tlr_geom(n, opts->tile, opts->max_rank).total;
    return 0;
  }
  if (opts && (opts->chol_mode < MVN_CHOL_ADAPTIVE || opts->chol_mode > MVN_CHOL_FP64))
    return fail(-2, "unknown chol_mode %d", opts->chol_mode);
  const size_t ld = padded(n);
  *bytes = align_up(sizeof(double) * ld * ld) + dense_header_bytes((int)ld) +
           align_up((size_t)elem_bytes_low(prec) * ld * ld);
  return 0;
}

int mvn_cholesky_workspace_bytes(int n, const mvn_options* opts, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (!bytes) return fail(-3, "bytes is NULL");
  *bytes = 0;
  if (is_tlr(opts)) {
    if (tlr_opts_check(opts)) return -2;
    *bytes = tlr_geom(n, opts->tile, opts->max_rank).ws_total;
  }
  return 0;
}

int mvn_prob_workspace_bytes(int n, int N, int S, const mvn_options* opts, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (N < 1) return fail(-2, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-3, "S must be >= 1 (got %d)", S);
  if (!bytes) return fail(-5, "bytes is NULL");
  const int prec = opts ? opts->precision : MVN_FP64;
  if (!prec_ok(prec)) return fail(-4, "unknown precision %d", prec);
  if (is_tlr(opts)) {
    // every tile at the rank stride: enough for any factor with these options
    if (tlr_opts_check(opts)) return -4;
    if (!tlr_rows_ok(opts)) return fail(-4, "sweep_rows must be 0, 64, 128 or 256 (got %d)", opts->sweep_rows);
    const TlrGeom G = tlr_geom(n, opts->tile, opts->max_rank);
    const long kmax = G.npanels * G.rs;
    const TlrProbLayout L = tlr_prob_layout(G.ld, G.nt, G.rs, N, S, tlr_sweep_rows(opts, (long)N * S));
    *bytes = L.fixed + L.dyn_bytes(kmax, kmax, L.grid, G.m);
    return 0;
  }
  if (!dense_rows_ok(opts))
    return fail(-4, "sweep_rows must be 0, 64, 128 or 32 (FP64) (got %d)", opts->sweep_rows);
  *bytes = prob_layout(n, N, S, prec, rows_opt(opts)).total;
  return 0;
}

int mvn_prob_workspace_bytes_factor(const mvn_factor* f, int N, int S, const mvn_options* opts, size_t* bytes,
                                    hipStream_t stream) {
  if (!f || !f->L || f->n < 1) return fail(-1, "invalid factor handle");
  if (!(f->flags & MVN_FACTOR_TLR)) return mvn_prob_workspace_bytes(f->n, N, S, opts, bytes);
  if (N < 1) return fail(-2, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-3, "S must be >= 1 (got %d)", S);
  if (!bytes) return fail(-5, "bytes is NULL");
  if (!f->ranks || f->tile < 128 || f->ld % f->tile != 0) return fail(-1, "invalid factor handle");
  if (!tlr_rows_ok(opts)) return fail(-4, "sweep_rows must be 0, 64, 128 or 256 (got %d)", opts->sweep_rows);
  std::vector<int> ranks;
  const hipError_t e = tlr_read_ranks(f, ranks, stream);
  if (e != hipSuccess) return hip_fail(e, "rank read-back");
  const int nt = f->ld / f->tile;
  const mvn::TlrTables T = mvn::build_tlr_tables(nt, f->rank_stride, ranks.data());
  const TlrProbLayout L =
      tlr_prob_layout(f->ld, nt, f->rank_stride, N, S, tlr_sweep_rows(opts, (long)N * S), is_compact(f));
  *bytes = L.fixed + L.dyn_bytes(T.ksum, T.kpad0[nt], L.grid, f->tile);
  return 0;
}

int mvn_prob_prefix_workspace_bytes(const mvn_factor* f, int N, int S, const mvn_options* opts, size_t* bytes,
                                    hipStream_t stream) {
  if (!f || !f->L || f->n < 1) return fail(-1, "invalid factor handle");
  if (N < 64) return fail(-2, "the nested-set sweep needs N >= 64 (got %d)", N);
  if (S < 1) return fail(-3, "S must be >= 1 (got %d)", S);
  if (!bytes) return fail(-5, "bytes is NULL");
  size_t rest = 0;
  const int rc = mvn_prob_workspace_bytes_factor(f, N, S, opts, &rest, stream);
  if (rc) return rc;
  const bool tlr = (f->flags & MVN_FACTOR_TLR) != 0;
  const int cols = tlr ? mvn::sweep_tile_cols()
                       : prefix_cols(opts ? opts->precision : MVN_FP64, rows_opt(opts), (long)N * S, f->n);
  *bytes = prefix_region(f->n, N, S, cols).total + rest;
  return 0;
}

int mvn_prob_prefix(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int N, int S,
                    uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes, double* d_prefix,
                    hipStream_t stream) {
  if (!f || !f->L || !f->info || f->n < 1) return fail(-1, "invalid factor handle");
  const bool tlr = (f->flags & MVN_FACTOR_TLR) != 0;
  if (tlr ? (f->tile < 128 || f->tile % 128 != 0 || f->ld % f->tile != 0 || f->ld < f->n || f->ld - f->n >= f->tile ||
             !f->U || !f->Vt || !f->ranks || f->rank_stride < 16 || f->rank_stride % 16 != 0)
          : f->ld != padded(f->n))
    return fail(-1, "invalid factor handle");
  if (!d_a) return fail(-2, "lower limits are NULL");
  if (!d_b) return fail(-3, "upper limits are NULL");
  if (N < 64) return fail(-5, "the nested-set sweep needs N >= 64 (got %d)", N);
  if (S < 1) return fail(-6, "S must be >= 1 (got %d)", S);
  if ((long)N * S > (long)INT32_MAX * 64) return fail(-5, "N*S too large");
  if (!opts) return fail(-8, "options are required");
  const int prec = opts->precision;
  if (!prec_ok(prec)) return fail(-8, "unknown precision %d", prec);
  if (tlr && prec != MVN_FP64) return fail(-8, "the TLR sweep is FP64");
  if (!tlr && prec != MVN_FP64 && (prec != f->precision || !f->L_low))
    return fail(-8, "the factor holds no operand copy for precision %d (built with %d)", prec, f->precision);
  if (tlr ? !tlr_rows_ok(opts) : !dense_rows_ok(opts))
    return fail(-8, "sweep_rows must be 0, 64, 128, 32 (FP64, dense) or 256 (TLR) (got %d)", opts->sweep_rows);
  const PrefixRegion R =
      prefix_region(f->n, N, S, tlr ? mvn::sweep_tile_cols() : prefix_cols(prec, rows_opt(opts), (long)N * S, f->n));
  if (!ws) return fail(-9, "workspace is NULL");
  if (ws_bytes < R.total) return fail(-10, "workspace too small: %zu < %zu", ws_bytes, R.total);
  if (!d_prefix) return fail(-11, "output is NULL");
  char* w = (char*)ws;
  double* part = (double*)(w + R.part);
  void* rest = w + R.total;
  const size_t rest_bytes = ws_bytes - R.total;
  const int* bad = nullptr;
  int rc;
  if (tlr) {
    rc = tlr_sweep_call(f, d_a, d_b, d_mu, N, S, seed, opts, rest, rest_bytes, nullptr, part, nullptr, stream, &bad);
  } else {
    const ProbLayout Lay = prob_layout(f->n, N, S, prec, rows_opt(opts), true);
    if (rest_bytes < Lay.total) return fail(-10, "workspace too small: %zu < %zu", ws_bytes, R.total + Lay.total);
    bad = (const int*)((char*)rest + Lay.bad);
    rc = dense_sweep(f, d_a, d_b, d_mu, N, S, seed, opts, rest, Lay, nullptr, part, nullptr, stream);
  }
  if (rc) return rc;
  const hipError_t e = mvn::launch_prefix_reduce(part, R.nchunks, R.cols, f->n, N, S, (double*)(w + R.lps), f->info,
                                                 bad, d_prefix, stream);
  if (e != hipSuccess) return hip_fail(e, "prefix reduce");
  return 0;
}

int mvn_mc_prefix_workspace_bytes(int n, int M, const mvn_options* opts, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (M < 1) return fail(-2, "M must be >= 1 (got %d)", M);
  if (!sweep_rows_ok(opts)) return fail(-3, "sweep_rows must be 0, 64 or 128 (got %d)", opts->sweep_rows);
  if (!bytes) return fail(-4, "bytes is NULL");
  *bytes = mc_layout(n, M, mc_rows(opts)).total;
  return 0;
}

int mvn_mc_prefix(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int M,
                  uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes, int* d_first, int64_t* d_count,
                  hipStream_t stream) {
  if (!f || !f->L || !f->info || f->n < 1) return fail(-1, "invalid factor handle");
  if (f->flags & MVN_FACTOR_TLR) return fail(-1, "the Monte Carlo check needs a dense factor");
  if (f->ld != padded(f->n)) return fail(-1, "invalid factor handle");
  if (!d_a) return fail(-2, "lower limits are NULL");
  if (!d_b) return fail(-3, "upper limits are NULL");
  if (M < 1) return fail(-5, "M must be >= 1 (got %d)", M);
  if (!sweep_rows_ok(opts)) return fail(-7, "sweep_rows must be 0, 64 or 128 (got %d)", opts->sweep_rows);
  const McLayout Lay = mc_layout(f->n, M, mc_rows(opts));
  if (!ws) return fail(-8, "workspace is NULL");
  if (ws_bytes < Lay.total) return fail(-9, "workspace too small: %zu < %zu", ws_bytes, Lay.total);
  if (!d_count) return fail(-11, "count output is NULL");
  char* w = (char*)ws;
  mvn::McArgs a{};
  a.L = f->L;
  a.ld = f->ld;
  a.n = f->n;
  a.a = d_a;
  a.b = d_b;
  a.mu = d_mu;
  a.seed = seed;
  a.M = M;
  a.yscr = (double*)(w + Lay.yscr);
  a.yslice = Lay.yslice;
  a.first = d_first;
  a.hist = (unsigned long long*)(w + Lay.hist);
  a.counter = (unsigned long long*)(w + Lay.counter);
  a.count = (long long*)d_count;
  a.info = f->info;
  a.grid = Lay.grid;
  a.rows = Lay.rows;
  const hipError_t e = mvn::launch_mc(a, stream);
  if (e != hipSuccess) return hip_fail(e, "Monte Carlo check");
  return 0;
}


int mvn_prob_grad_workspace_bytes(int n, int N, int S, const mvn_options* opts, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (N < 1) return fail(-2, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-3, "S must be >= 1 (got %d)", S);
  if (!bytes) return fail(-5, "bytes is NULL");
  (void)opts;
  *bytes = grad_layout(n, N, S).total;
  return 0;
}

namespace {

// mvn_cholesky, with Sigma optionally read in the order d_perm (device;
// perm_bad: the flag of its device check).
int cholesky_impl(int n, const double* d_sigma, int ld_sigma, const int64_t* d_perm, const int* perm_bad,
                  const double* d_locs, const mvn_matern* kern, const mvn_options* opts, void* factor_buf,
                  size_t factor_bytes, void* ws, size_t ws_bytes, mvn_factor* out, hipStream_t stream) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (d_sigma && ld_sigma < n) return fail(-3, "ld_sigma %d < n %d", ld_sigma, n);
  if (!d_sigma) {
    if (!d_locs) return fail(-4, "either sigma or locations are required");
    if (!kern) return fail(-5, "kernel parameters are required with locations");
    if (!mvn::matern_ok(kern->sigma2, kern->beta, kern->nu, kern->nugget))
      return fail(-5, "Matern parameters need sigma2 > 0, beta > 0, 0 < nu <= 20, nugget >= 0 (got %g, %g, %g, %g)",
                  kern->sigma2, kern->beta, kern->nu, kern->nugget);
  }
  if (!opts) return fail(-6, "options are required");
  int bad_tile = 0;
  if (!opts_ok(opts, &bad_tile)) return fail(-6, "tile must be >= 16 and a multiple of 4 (got %d)", opts->tile);
  if (!prec_ok(opts->precision)) return fail(-6, "unknown precision %d", opts->precision);
  if (is_tlr(opts)) {
    if (tlr_opts_check(opts)) return -6;
    const TlrGeom G = tlr_geom(n, opts->tile, opts->max_rank);
    if (!factor_buf) return fail(-7, "factor buffer is NULL");
    if (factor_bytes < G.total) return fail(-8, "factor buffer too small: %zu < %zu", factor_bytes, G.total);
    if (!ws) return fail(-9, "workspace is NULL (the TLR factorisation needs %zu bytes)", G.ws_total);
    if (ws_bytes < G.ws_total) return fail(-10, "workspace too small: %zu < %zu", ws_bytes, G.ws_total);
    if (!out) return fail(-11, "out is NULL");
    char* fb = (char*)factor_buf;
    char* w = (char*)ws;
    memset(out, 0, sizeof *out);
    out->n = n;
    out->ld = G.ld;
    out->precision = MVN_FP64;
    out->flags = MVN_FACTOR_TLR;
    out->L = (double*)(fb + G.tiles);
    out->info = (int*)(fb + G.info);
    out->L_low = nullptr;
    out->tile = G.m;
    out->rank_stride = G.rs;
    out->U = (double*)(fb + G.U);
    out->Vt = (double*)(fb + G.Vt);
    out->ranks = (int*)(fb + G.ranks);
    out->tlr_eps = opts->tlr_eps;
    out->max_rank = opts->max_rank;
    hipError_t e = mvn::launch_tlr_build(n, G.m, G.nt, d_sigma, ld_sigma, d_perm, perm_bad, d_locs, matern_of(kern), out->L,
                                         out->info, stream);
    if (e != hipSuccess) return hip_fail(e, "tlr build");
    mvn::TlrCholArgs a{};
    a.tiles = out->L;
    a.U = out->U;
    a.Vt = out->Vt;
    a.ranks = out->ranks;
    a.info = out->info;
    a.local_info = (int*)(w + G.ws_local);
    a.WT = (double*)(w + G.ws_wt);
    a.T = (double*)(w + G.ws_t);
    a.rc_scratch = G.rc_grid > 0 ? (double*)(w + G.ws_rc) : nullptr;
    a.rc_grid = G.rc_grid;
    a.m = G.m;
    a.nt = G.nt;
    a.rs = G.rs;
    a.rcap = opts->max_rank;
    a.eps = opts->tlr_eps;
    e = mvn::launch_tlr_cholesky(a, stream);
    if (e != hipSuccess) return hip_fail(e, "tlr cholesky");
    return 0;
  }
  size_t need = 0;
  mvn_factor_bytes(n, opts, &need);
  if (!factor_buf) return fail(-7, "factor buffer is NULL");
  if (factor_bytes < need) return fail(-8, "factor buffer too small: %zu < %zu", factor_bytes, need);
  if (!out) return fail(-11, "out is NULL");
  if (opts->chol_mode < MVN_CHOL_ADAPTIVE || opts->chol_mode > MVN_CHOL_FP64)
    return fail(-6, "unknown chol_mode %d", opts->chol_mode);
  const int ld = padded(n);
  double* L = (double*)factor_buf;
  char* hdr = (char*)factor_buf + align_up(sizeof(double) * (size_t)ld * ld);
  int* info = (int*)hdr;
  void* low = opts->precision == MVN_FP64 ? nullptr : hdr + dense_header_bytes(ld);
  out->n = n;
  out->ld = ld;
  out->precision = opts->precision;
  out->flags = 0;
  out->L = L;
  out->info = info;
  out->L_low = low;
  out->tile = 0;
  out->rank_stride = 0;
  out->U = nullptr;
  out->Vt = nullptr;
  out->ranks = nullptr;
  out->tlr_eps = 0;
  out->max_rank = 0;
  out->chol_mode = opts->precision == MVN_FP64 ? MVN_CHOL_FP64 : opts->chol_mode;
  out->update_counts = (unsigned long long*)(hdr + 16);
  hipError_t e = mvn::launch_clear_u64(out->update_counts, 3, stream);
  if (e != hipSuccess) return hip_fail(e, "counter clear");
  e = mvn::launch_build_matrix(n, ld, d_sigma, ld_sigma, d_perm, perm_bad, d_locs, matern_of(kern), L, info, stream);
  if (e != hipSuccess) return hip_fail(e, "build_matrix");
  if (opts->precision == MVN_FP64) {
    e = mvn::launch_cholesky_f64(ld, opts->tile, L, info, stream);
  } else {
    mvn::LpMap map{(double*)(hdr + 64), (double*)(hdr + 8), out->update_counts,
                   opts->chol_tol > 0 ? opts->chol_tol : 1e-9};
    e = mvn::launch_cholesky_lp(opts->precision, ld, opts->tile, L, info, low, stream,
                                opts->chol_mode == MVN_CHOL_ADAPTIVE ? &map : nullptr,
                                opts->chol_mode == MVN_CHOL_FP64);
  }
  if (e != hipSuccess) return hip_fail(e, "cholesky");
  return 0;
}

// Layout of a posterior workspace: observation indices, then the bordered
// matrix (observations padded to the tile, sites, the data row).
struct PostLayout {
  size_t obs, B, total;
  long mpad, ld;
};

PostLayout post_layout(int n, int m, int tile) {
  PostLayout P{};
  P.mpad = ((long)m + tile - 1) / tile * tile;
  P.ld = (P.mpad + n + 1 + 127) / 128 * 128;
  size_t off = 0;
  P.obs = off; off = align_up(off + sizeof(int));  // the observation index check's flag
  P.B = off; off = align_up(off + sizeof(double) * (size_t)P.ld * (size_t)P.ld);
  P.total = off;
  return P;
}

}  // namespace

int mvn_cholesky(int n, const double* d_sigma, int ld_sigma, const double* d_locs, const mvn_matern* kern,
                 const mvn_options* opts, void* factor_buf, size_t factor_bytes, void* ws, size_t ws_bytes,
                 mvn_factor* out, hipStream_t stream) {
  return cholesky_impl(n, d_sigma, ld_sigma, nullptr, nullptr, d_locs, kern, opts, factor_buf, factor_bytes, ws,
                       ws_bytes, out, stream);
}

int mvn_cholesky_permuted_workspace_bytes(int n, const mvn_options* opts, size_t* bytes) {
  if (!bytes) return fail(-3, "bytes is NULL");
  size_t base = 0;
  const int rc = mvn_cholesky_workspace_bytes(n, opts, &base);
  if (rc) return rc;
  // the permutation check: a flag and one int per site
  *bytes = align_up(base) + kAlign + align_up(sizeof(int) * (size_t)n);
  return 0;
}

int mvn_cholesky_permuted(int n, const double* d_sigma, int ld_sigma, const int64_t* d_perm, const mvn_options* opts,
                          void* factor_buf, size_t factor_bytes, void* ws, size_t ws_bytes, mvn_factor* out,
                          hipStream_t stream) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (!d_sigma) return fail(-2, "sigma is NULL");
  if (ld_sigma < n) return fail(-3, "ld_sigma %d < n %d", ld_sigma, n);
  if (!d_perm) return fail(-4, "perm is NULL");
  if (!opts) return fail(-5, "options are required");
  int bad_tile = 0;
  if (!opts_ok(opts, &bad_tile)) return fail(-5, "tile must be >= 16 and a multiple of 4 (got %d)", opts->tile);
  if (!prec_ok(opts->precision)) return fail(-5, "unknown precision %d", opts->precision);
  if (is_tlr(opts) && tlr_opts_check(opts)) return -5;
  size_t base = 0, need = 0, fbytes = 0;
  if (mvn_cholesky_workspace_bytes(n, opts, &base) || mvn_cholesky_permuted_workspace_bytes(n, opts, &need) ||
      mvn_factor_bytes(n, opts, &fbytes))
    return -5;  // the options are bad; the message is set
  if (!factor_buf) return fail(-6, "factor buffer is NULL");
  if (factor_bytes < fbytes) return fail(-7, "factor buffer too small: %zu < %zu", factor_bytes, fbytes);
  if (!ws) return fail(-8, "workspace is NULL");
  if (ws_bytes < need) return fail(-9, "workspace too small: %zu < %zu", ws_bytes, need);
  if (!out) return fail(-10, "out is NULL");
  int* flag = (int*)((char*)ws + align_up(base));
  int* seen = (int*)((char*)ws + align_up(base) + kAlign);
  const hipError_t e = mvn::launch_index_check(d_perm, n, n, seen, flag, stream);
  if (e != hipSuccess) return hip_fail(e, "permutation check");
  // every argument is valid here, so the shared implementation only enqueues
  return cholesky_impl(n, d_sigma, ld_sigma, d_perm, flag, nullptr, nullptr, opts, factor_buf, factor_bytes, ws, base,
                       out, stream);
}

int mvn_posterior_workspace_bytes(int n, int m, const mvn_options* opts, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (m < 1) return fail(-2, "m must be >= 1 (got %d)", m);
  int bad_tile = 0;
  if (!opts || !opts_ok(opts, &bad_tile)) return fail(-3, "options with a valid tile are required");
  if (!bytes) return fail(-4, "bytes is NULL");
  *bytes = post_layout(n, m, opts->tile).total;
  return 0;
}

int mvn_posterior(int n, const double* d_locs, const double* d_mu, int m, const int64_t* d_obs, const double* d_y,
                  const mvn_matern* kern, double noise_var, const mvn_options* opts, void* ws, size_t ws_bytes,
                  double* d_mu_post, double* d_var_post, int* d_info, double** sigma_post, int* ld_sigma_post,
                  hipStream_t stream) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (!d_locs) return fail(-2, "locations are NULL");
  if (m < 1) return fail(-4, "m must be >= 1 (got %d)", m);
  if (!d_obs) return fail(-5, "observation indices are NULL");
  if (!d_y) return fail(-6, "observations are NULL");
  if (!kern || !mvn::matern_ok(kern->sigma2, kern->beta, kern->nu, kern->nugget))
    return fail(-7, "Matern parameters need sigma2 > 0, beta > 0, 0 < nu <= 20, nugget >= 0");
  if (!(noise_var > 0) || !isfinite(noise_var)) return fail(-8, "noise variance must be > 0 (got %g)", noise_var);
  int bad_tile = 0;
  if (!opts || !opts_ok(opts, &bad_tile)) return fail(-9, "options with a valid tile are required");
  if (opts->precision != MVN_FP64) return fail(-9, "the posterior is computed in FP64");
  const PostLayout P = post_layout(n, m, opts->tile);
  if ((long)P.ld > INT32_MAX) return fail(-1, "n + m too large");
  if (!ws) return fail(-10, "workspace is NULL");
  if (ws_bytes < P.total) return fail(-11, "workspace too small: %zu < %zu", ws_bytes, P.total);
  if (!d_info) return fail(-14, "info is NULL");
  char* w = (char*)ws;
  mvn::PosteriorArgs a{};
  a.obs_bad = (const int*)(w + P.obs);
  a.B = (double*)(w + P.B);
  a.ld = P.ld;
  a.n = n;
  a.m = m;
  a.mpad = P.mpad;
  a.obs = d_obs;
  a.locs = d_locs;
  a.y = d_y;
  a.mu = d_mu;
  a.mk = matern_of(kern);
  a.noise_var = noise_var;
  a.info = d_info;
  const hipError_t e = mvn::launch_posterior(a, opts->tile, d_mu_post, d_var_post, stream);
  if (e != hipSuccess) return hip_fail(e, "posterior");
  if (sigma_post) *sigma_post = a.B + P.mpad * P.ld + P.mpad;
  if (ld_sigma_post) *ld_sigma_post = (int)P.ld;
  return 0;
}

int mvn_prob(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int N,
             int S, uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes, double* d_out,
             double* d_ell, hipStream_t stream) {
  if (!f || !f->L || !f->info || f->n < 1) return fail(-1, "invalid factor handle");
  const bool tlr = (f->flags & MVN_FACTOR_TLR) != 0;
  if (tlr ? (f->tile < 128 || f->tile % 128 != 0 || f->ld % f->tile != 0 || f->ld < f->n || f->ld - f->n >= f->tile ||
             !f->U || !f->Vt || !f->ranks || f->rank_stride < 16 || f->rank_stride % 16 != 0)
          : f->ld != padded(f->n))
    return fail(-1, "invalid factor handle");
  if (!d_a) return fail(-2, "lower limits are NULL");
  if (!d_b) return fail(-3, "upper limits are NULL");
  if (N < 1) return fail(-5, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-6, "S must be >= 1 (got %d)", S);
  if ((long)N * S > (long)INT32_MAX * 64) return fail(-5, "N*S too large");
  if (!opts) return fail(-8, "options are required");
  const int prec = opts->precision;
  if (!prec_ok(prec)) return fail(-8, "unknown precision %d", prec);
  if (tlr) {
    if (prec != MVN_FP64) return fail(-8, "the TLR sweep is FP64");
    if (!tlr_rows_ok(opts)) return fail(-8, "sweep_rows must be 0, 64, 128 or 256 (got %d)", opts->sweep_rows);
    if (!ws) return fail(-9, "workspace is NULL");
    if (!d_out) return fail(-11, "output is NULL");
    return tlr_sweep_call(f, d_a, d_b, d_mu, N, S, seed, opts, ws, ws_bytes, d_ell, nullptr, d_out, stream, nullptr);
  }
  if (prec != MVN_FP64 && (prec != f->precision || !f->L_low))
    return fail(-8, "the factor holds no operand copy for precision %d (built with %d)", prec, f->precision);
  if (!dense_rows_ok(opts))
    return fail(-8, "sweep_rows must be 0, 64, 128 or 32 (FP64) (got %d)", opts->sweep_rows);
  const ProbLayout Lay = prob_layout(f->n, N, S, prec, rows_opt(opts));
  if (!ws) return fail(-9, "workspace is NULL");
  if (ws_bytes < Lay.total) return fail(-10, "workspace too small: %zu < %zu", ws_bytes, Lay.total);
  if (!d_out) return fail(-11, "output is NULL");
  return dense_sweep(f, d_a, d_b, d_mu, N, S, seed, opts, ws, Lay, d_ell, nullptr, d_out, stream);
}

size_t exceed_ws(int n, size_t* key, size_t* idx, size_t* bad) {
  const size_t npad = (size_t)mvn::exceedance_npad(n);
  size_t off = 0;
  *key = off; off = align_up(off + sizeof(double) * npad);
  *idx = off; off = align_up(off + sizeof(int64_t) * npad);
  *bad = off; off = align_up(off + sizeof(int));
  return off;
}

int mvn_exceedance_order_workspace_bytes(int n, size_t* bytes) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (!bytes) return fail(-2, "bytes is NULL");
  size_t k, i, b;
  *bytes = exceed_ws(n, &k, &i, &b);
  return 0;
}

int mvn_exceedance_order(int n, const double* d_mu, const double* d_var, double u, int64_t* d_perm, double* d_p,
                         void* ws, size_t ws_bytes, hipStream_t stream) {
  if (n < 1) return fail(-1, "n must be >= 1 (got %d)", n);
  if (!d_mu) return fail(-2, "mean is NULL");
  if (!d_var) return fail(-3, "variances are NULL");
  if (!isfinite(u)) return fail(-4, "u must be finite");
  if (!d_perm) return fail(-5, "output permutation is NULL");
  size_t k, i, b;
  const size_t need = exceed_ws(n, &k, &i, &b);
  if (!ws) return fail(-7, "workspace is NULL");
  if (ws_bytes < need) return fail(-8, "workspace too small: %zu < %zu", ws_bytes, need);
  char* w = (char*)ws;
  const hipError_t e = mvn::launch_exceedance_order(n, d_mu, d_var, u, (double*)(w + k), (int64_t*)(w + i),
                                                    (int*)(w + b), d_p, d_perm, stream);
  if (e != hipSuccess) return hip_fail(e, "exceedance order");
  return 0;
}

// Compact TLR factor: info | ranks | diagonal tiles | V' rows (ksum + 128) x m |
// U columns m x kpad | the sweep's index tables (built there once, by the
// same kernel as per call, to place the packed operands).
struct TlrCompactLayout {
  size_t info, ranks, diag, vpack, upack, kk, zcol, kpad0, kval, vrow0, ucol0, zdst, hdr, flag, total;
};

TlrCompactLayout tlr_compact_layout(int nt, int m, int rs, long ksum, long kpad) {
  TlrCompactLayout L{};
  const size_t np = (size_t)nt * (nt - 1) / 2, np1 = np > 0 ? np : 1;
  size_t off = 0;
  L.info = off; off = align_up(off + sizeof(int));
  L.ranks = off; off = align_up(off + sizeof(int) * np1);
  L.diag = off; off = align_up(off + sizeof(double) * (size_t)nt * m * m);
  L.vpack = off;  // the tables kernel puts U at the next 256-byte boundary after V'
  L.upack = off + align_up(8 * (size_t)(ksum + 128) * m);
  off = align_up(L.upack + 8 * (size_t)m * (size_t)(kpad > 0 ? kpad : 1));
  L.kk = off; off = align_up(off + sizeof(int) * np1);
  L.zcol = off; off = align_up(off + sizeof(long) * (nt + 1));
  L.kpad0 = off; off = align_up(off + sizeof(long) * (nt + 1));
  L.kval = off; off = align_up(off + sizeof(int) * nt);
  L.vrow0 = off; off = align_up(off + sizeof(long) * np1);
  L.ucol0 = off; off = align_up(off + sizeof(long) * np1);
  L.zdst = off; off = align_up(off + sizeof(long) * np1 * rs);
  L.hdr = off; off = align_up(off + sizeof(mvn::TlrSweepHdr));
  L.flag = off; off = align_up(off + sizeof(int));
  L.total = off;
  return L;
}

bool full_tlr_ok(const mvn_factor* f) {
  return f && (f->flags & MVN_FACTOR_TLR) && !is_compact(f) && f->L && f->info && f->n >= 1 && f->tile >= 128 &&
         f->tile % 128 == 0 && f->ld % f->tile == 0 && f->ld >= f->n && f->U && f->Vt && f->ranks &&
         f->rank_stride >= 16 && f->rank_stride % 16 == 0;
}

int tlr_compact_plan(const mvn_factor* f, TlrCompactLayout* L, hipStream_t stream) {
  std::vector<int> ranks;
  const hipError_t e = tlr_read_ranks(f, ranks, stream);
  if (e != hipSuccess) return hip_fail(e, "rank read-back");
  const int nt = f->ld / f->tile;
  const mvn::TlrTables T = mvn::build_tlr_tables(nt, f->rank_stride, ranks.data());
  *L = tlr_compact_layout(nt, f->tile, f->rank_stride, T.ksum, T.kpad0[nt]);
  return 0;
}

int mvn_tlr_compact_bytes(const mvn_factor* f, size_t* bytes, hipStream_t stream) {
  if (!full_tlr_ok(f)) return fail(-1, "not a full TLR factor handle");
  if (!bytes) return fail(-2, "bytes is NULL");
  TlrCompactLayout L;
  const int rc = tlr_compact_plan(f, &L, stream);
  if (rc) return rc;
  *bytes = L.total;
  return 0;
}

int mvn_tlr_compact(const mvn_factor* f, void* d_buf, size_t bytes, mvn_factor* out, hipStream_t stream) {
  if (!full_tlr_ok(f)) return fail(-1, "not a full TLR factor handle");
  if (!d_buf) return fail(-2, "buffer is NULL");
  if (!out) return fail(-4, "output handle is NULL");
  TlrCompactLayout L;
  const int rc = tlr_compact_plan(f, &L, stream);
  if (rc) return rc;
  if (bytes < L.total) return fail(-3, "buffer too small: %zu < %zu", bytes, L.total);
  const int m = f->tile, nt = f->ld / f->tile, rs = f->rank_stride;
  const int np = nt * (nt - 1) / 2;
  char* b = (char*)d_buf;
  hipError_t e = hipMemcpyAsync(b + L.info, f->info, sizeof(int), hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && np > 0)
    e = hipMemcpyAsync(b + L.ranks, f->ranks, sizeof(int) * np, hipMemcpyDeviceToDevice, stream);
  for (int i = 0; i < nt && e == hipSuccess; ++i)
    e = hipMemcpyAsync(b + L.diag + sizeof(double) * (size_t)i * m * m,
                       f->L + ((size_t)i * (i + 1) / 2 + i) * (size_t)m * m, sizeof(double) * (size_t)m * m,
                       hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "compact copy");
  mvn::TlrTableArgs tb{};
  tb.ranks = f->ranks;
  tb.nt = nt;
  tb.rs = rs;
  tb.m = m;
  tb.ext_pack = 0;  // the packed operands at the header's offsets from the compact V' start
  tb.yslice = 0;
  tb.grid_max = 1;
  tb.dyn_bytes = (size_t)1 << 62;  // only sizes the (unused) sweep grid, which stays 1
  tb.kk = (int*)(b + L.kk);
  tb.zcol = (long*)(b + L.zcol);
  tb.kpad0 = (long*)(b + L.kpad0);
  tb.kval = (int*)(b + L.kval);
  tb.vrow0 = (long*)(b + L.vrow0);
  tb.ucol0 = (long*)(b + L.ucol0);
  tb.zdst = (long*)(b + L.zdst);
  tb.hdr = (mvn::TlrSweepHdr*)(b + L.hdr);
  tb.bad = (int*)(b + L.flag);  // written only when no sweep workgroup fits, never here
  e = mvn::launch_tlr_tables(tb, stream);
  if (e != hipSuccess) return hip_fail(e, "tlr tables");
  mvn::TlrPackArgs pa{};
  pa.U = f->U;
  pa.Vt = f->Vt;
  pa.m = m;
  pa.rs = rs;
  pa.np = np;
  pa.kk = tb.kk;
  pa.vrow0 = tb.vrow0;
  pa.ucol0 = tb.ucol0;
  pa.kpad0 = tb.kpad0;
  pa.kval = tb.kval;
  pa.hdr = tb.hdr;
  pa.dyn = b + L.vpack;
  e = mvn::launch_tlr_pack(pa, stream);
  if (e != hipSuccess) return hip_fail(e, "tlr pack");
  mvn_factor c = *f;
  c.flags = MVN_FACTOR_TLR | MVN_FACTOR_TLR_COMPACT;
  c.L = (double*)(b + L.diag);
  c.info = (int*)(b + L.info);
  c.U = (double*)(b + L.upack);
  c.Vt = (double*)(b + L.vpack);
  c.ranks = (int*)(b + L.ranks);
  c.L_low = nullptr;
  c.update_counts = nullptr;
  *out = c;
  return 0;
}

int mvn_tlr_dense_bytes(const mvn_factor* f, size_t* bytes) {
  if (!bytes) return fail(-2, "bytes is NULL");
  if (!f || !(f->flags & MVN_FACTOR_TLR) || is_compact(f) || f->n < 1) return fail(-1, "not a full TLR factor handle");
  const size_t ld = (size_t)padded(f->n);
  *bytes = sizeof(double) * ld * ld;
  return 0;
}

int mvn_tlr_dense(const mvn_factor* f, void* d_buf, size_t bytes, mvn_factor* out, hipStream_t stream) {
  if (!f || !(f->flags & MVN_FACTOR_TLR) || is_compact(f) || !f->L || !f->info || f->n < 1 || f->tile < 128 || f->tile % 128 != 0 ||
      f->ld % f->tile != 0 || f->ld < f->n || !f->U || !f->Vt || !f->ranks || f->rank_stride < 16 ||
      f->rank_stride % 16 != 0)
    return fail(-1, "not a TLR factor handle");
  if (!d_buf) return fail(-2, "buffer is NULL");
  const long ld = padded(f->n);
  if (bytes < sizeof(double) * (size_t)ld * (size_t)ld)
    return fail(-3, "buffer too small: %zu < %zu", bytes, sizeof(double) * (size_t)ld * (size_t)ld);
  if (!out) return fail(-4, "output handle is NULL");
  const hipError_t e = mvn::launch_tlr_expand(f->n, f->tile, f->ld / f->tile, f->rank_stride, f->L, f->U, f->Vt,
                                              f->ranks, (double*)d_buf, ld, stream);
  if (e != hipSuccess) return hip_fail(e, "TLR expansion");
  mvn_factor d{};
  d.n = f->n;
  d.ld = (int)ld;
  d.precision = MVN_FP64;
  d.flags = 0;
  d.L = (double*)d_buf;
  d.info = f->info;
  d.chol_mode = MVN_CHOL_FP64;
  *out = d;
  return 0;
}

// ---------------------------------------------------------------- no-allocation variant
}  // extern "C"

namespace {

// The device memory of mvn_prob_static: one file-scope array per GPU, held
// until the process ends.  In host code `scratch` names a host-side stand-in;
// its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticBytes = (size_t)256 << 20;
constexpr int kStaticMaxN = 1 << 17;  // lattice entries kept at the front of scratch
constexpr size_t kStaticLat = (size_t)kStaticMaxN * sizeof(uint64_t);
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
unsigned char* g_static_ptr[kMaxDevices] = {};

// Host copy of the lattice table for kStaticMaxN dimensions, built once in
// static storage (no allocation): the sieve runs over a fixed bound above
// p_131072 = 1742537.
constexpr size_t kStaticSieve = 1800000;
uint8_t g_static_comp[kStaticSieve];
uint64_t g_static_lat[kStaticMaxN];
bool g_static_lat_ready = false;

bool static_lattice_build() {
  int cnt = 0;
  for (size_t v = 2; v < kStaticSieve && cnt < kStaticMaxN; ++v) {
    if (g_static_comp[v]) continue;
    g_static_lat[cnt++] = frac_sqrt_2p64(v);
    for (size_t m = v * v; m < kStaticSieve; m += v) g_static_comp[m] = 1;
  }
  return cnt == kStaticMaxN;
}

// Device address of this device's scratch (set up on the first call on the
// device: symbol address, then the lattice table copied to its front).
int static_scratch(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(-1, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    if (!g_static_lat_ready) {
      if (!static_lattice_build()) return fail(-1, "could not build the lattice table");
      g_static_lat_ready = true;
    }
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    e = hipMemcpy(ptr, g_static_lat, kStaticLat, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "lattice copy to scratch");
    g_static_ptr[dev] = (unsigned char*)ptr;
  }
  *out = g_static_ptr[dev];
  return 0;
}

}  // namespace

extern "C" {

int mvn_prob_static(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu, int N, int S,
                    uint64_t seed, const mvn_options* opts, double* d_out, double* d_ell, hipStream_t stream) {
  if (!f || !f->L || !f->info || f->n < 1) return fail(-1, "invalid factor handle");
  if (f->flags & MVN_FACTOR_TLR) return fail(-1, "mvn_prob_static takes dense factors");
  if (f->ld != padded(f->n)) return fail(-1, "invalid factor handle");
  if (f->n > kStaticMaxN) return fail(-1, "n = %d exceeds the static limit %d", f->n, kStaticMaxN);
  if (!d_a) return fail(-2, "lower limits are NULL");
  if (!d_b) return fail(-3, "upper limits are NULL");
  if (N < 1) return fail(-5, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-6, "S must be >= 1 (got %d)", S);
  if ((long)N * S > (long)INT32_MAX * 64) return fail(-5, "N*S too large");
  if (!opts) return fail(-8, "options are required");
  const int prec = opts->precision;
  if (!prec_ok(prec)) return fail(-8, "unknown precision %d", prec);
  if (prec != MVN_FP64 && (prec != f->precision || !f->L_low))
    return fail(-8, "the factor holds no operand copy for precision %d (built with %d)", prec, f->precision);
  if (!dense_rows_ok(opts))
    return fail(-8, "sweep_rows must be 0, 64, 128 or 32 (FP64) (got %d)", opts->sweep_rows);
  if (!d_out) return fail(-9, "output is NULL");
  const int rows = sweep_rows(opts);
  const int kind = sweep_kind(prec, rows_opt(opts), false, (long)N * S, f->n);
  // as many persistent workgroups as the scratch holds
  const ProbLayout one = prob_layout_ld(padded(f->n), N, S, prec, 0, rows, kind, 1);
  const size_t per = align_up((size_t)mvn::sweep_elem_bytes(prec) * (size_t)one.yslice);
  const size_t avail = kStaticBytes - kStaticLat;
  if (one.total > avail)
    return fail(-5, "problem needs %zu bytes of scratch, the static limit is %zu (n = %d, N*S = %ld)", one.total,
                avail, f->n, (long)N * S);
  const int gcap = (int)std::min<size_t>((avail - one.total) / per + 1, (size_t)INT32_MAX);
  const ProbLayout Lay = prob_layout_ld(padded(f->n), N, S, prec, 0, rows, kind, gcap);
  unsigned char* base = nullptr;
  const int rc = static_scratch(&base);
  if (rc) return rc;
  return dense_sweep(f, d_a, d_b, d_mu, N, S, seed, opts, base + kStaticLat, Lay, d_ell, nullptr, d_out, stream,
                     (const uint64_t*)base);
}

int mvn_prob_grad(const mvn_factor* f, const double* d_a, const double* d_b, const double* d_mu,
                  int N, int S, uint64_t seed, const mvn_options* opts, void* ws, size_t ws_bytes,
                  double* d_out, double* d_da, double* d_db, double* d_dmu, hipStream_t stream) {
  if (!f || !f->L || !f->info || f->n < 1 || f->ld != padded(f->n))
    return fail(-1, "invalid factor handle");
  if (f->flags & MVN_FACTOR_TLR) return fail(-1, "the adjoint sweep needs a dense factor");
  if (!d_a) return fail(-2, "lower limits are NULL");
  if (!d_b) return fail(-3, "upper limits are NULL");
  if (N < 1) return fail(-5, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-6, "S must be >= 1 (got %d)", S);
  if (!opts) return fail(-8, "options are required");
  const int prec = opts->precision;
  if (!prec_ok(prec)) return fail(-8, "unknown precision %d", prec);
  if (prec != MVN_FP64 && (prec != f->precision || !f->L_low))
    return fail(-8, "the factor holds no operand copy for precision %d (built with %d)", prec, f->precision);
  const int n = f->n;
  const GradLayout Lay = grad_layout(n, N, S);
  if (!ws) return fail(-9, "workspace is NULL");
  if (ws_bytes < Lay.total) return fail(-10, "workspace too small: %zu < %zu", ws_bytes, Lay.total);
  if (!d_out) return fail(-11, "output is NULL");
  const uint64_t* lat = lattice_table(n);
  if (!lat) return fail(-1, "could not build the lattice table for n = %d", n);
  char* w = (char*)ws;
  double* at = (double*)(w + Lay.at);
  double* bt = (double*)(w + Lay.bt);
  uint64_t* dlat = (uint64_t*)(w + Lay.lat);
  double* ell = (double*)(w + Lay.ell);
  double* part = (double*)(w + Lay.part);
  int* bad = (int*)(w + Lay.bad);
  hipError_t e = hipMemcpyAsync(dlat, lat, sizeof(uint64_t) * n, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "lattice copy");
  e = mvn::launch_prob_setup(n, f->ld, d_a, d_b, d_mu, at, bt, bad, stream);
  if (e != hipSuccess) return hip_fail(e, "setup");
  mvn::GradArgs ga{};
  ga.L = f->L;
  ga.Llow = prec == MVN_FP64 ? (const void*)f->L : f->L_low;
  ga.prec = prec;
  ga.ld = f->ld;
  ga.n = n;
  ga.at = at;
  ga.bt = bt;
  ga.lattice = dlat;
  ga.seed = seed;
  ga.N = N;
  ga.S = S;
  ga.periodize = opts->periodize ? 1 : 0;
  ga.yscr = (double*)(w + Lay.yscr);
  ga.sfw = (double*)(w + Lay.sfw);
  ga.sbar = (double*)(w + Lay.sbar);
  ga.ell = ell;
  ga.gpart = (double*)(w + Lay.gpart);
  ga.mz = (double*)(w + Lay.mz);
  ga.grid = Lay.grid;
  e = mvn::launch_grad(ga, f->info, bad, (double*)(w + Lay.scale), d_da, d_db, d_dmu, stream);
  if (e != hipSuccess) return hip_fail(e, "adjoint sweep");
  e = mvn::launch_reduce(ell, N, S, part, f->info, bad, d_out, stream);
  if (e != hipSuccess) return hip_fail(e, "reduce");
  return 0;
}

int mvn_batch_plan_bytes(int count, size_t* bytes) {
  if (count < 1) return fail(-1, "count must be >= 1 (got %d)", count);
  if (!bytes) return fail(-2, "bytes is NULL");
  *bytes = batch_plan_bytes(count);
  return 0;
}

int mvn_batch_plan(int count, const int* n_p, int N, int S, const mvn_options* opts, void* plan,
                   size_t plan_bytes, size_t* factor_bytes, size_t* ws_bytes) {
  if (count < 1) return fail(-1, "count must be >= 1 (got %d)", count);
  if (!n_p) return fail(-2, "sizes are NULL");
  if (N < 1) return fail(-3, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-4, "S must be >= 1 (got %d)", S);
  const int prec = opts ? opts->precision : MVN_FP64;
  if (!prec_ok(prec)) return fail(-5, "unknown precision %d", prec);
  BatchPlan P;
  if (!batch_plan_host(count, n_p, P)) return fail(-2, "every problem needs n >= 1");
  if (plan) {
    if (plan_bytes < batch_plan_bytes(count)) return fail(-7, "plan buffer too small");
    memcpy(plan, P.desc.data(), sizeof(mvn::BatchDesc) * count);
    memcpy((char*)plan + align_up(sizeof(mvn::BatchDesc) * (size_t)count), P.order.data(), sizeof(int) * count);
  }
  if (!sweep_rows_ok(opts)) return fail(-5, "sweep_rows must be 0, 64 or 128 (got %d)", opts->sweep_rows);
  if (factor_bytes) *factor_bytes = batch_factor_bytes(P, prec);
  if (ws_bytes) *ws_bytes = batch_ws(P, count, N, S, prec, sweep_rows(opts)).total;
  return 0;
}

int mvn_prob_batch(int count, const int* n_p, const void* d_plan, const int64_t* d_idx, const double* d_locs,
                   const mvn_matern* kern, const double* d_a, const double* d_b, const double* d_mu, int N, int S,
                   uint64_t seed, const mvn_options* opts, void* factor_buf, size_t factor_bytes, void* ws,
                   size_t ws_bytes, double* d_out, int* d_info, hipStream_t stream) {
  if (count < 1) return fail(-1, "count must be >= 1 (got %d)", count);
  if (!n_p) return fail(-2, "sizes are NULL");
  if (!d_plan) return fail(-3, "plan is NULL");
  if (!d_idx) return fail(-4, "location indices are NULL");
  if (!d_locs) return fail(-5, "locations are NULL");
  if (!kern || !mvn::matern_ok(kern->sigma2, kern->beta, kern->nu, kern->nugget))
    return fail(-6, "Matern parameters need sigma2 > 0, beta > 0, 0 < nu <= 20, nugget >= 0");
  if (!d_a) return fail(-7, "lower limits are NULL");
  if (!d_b) return fail(-8, "upper limits are NULL");
  if (N < 1) return fail(-10, "N must be >= 1 (got %d)", N);
  if (S < 1) return fail(-11, "S must be >= 1 (got %d)", S);
  if (!opts) return fail(-13, "options are required");
  const int prec = opts->precision;
  if (!prec_ok(prec)) return fail(-13, "unknown precision %d", prec);
  if (is_tlr(opts)) return fail(-13, "batched problems use dense factors (tlr_eps must be <= 0)");
  BatchPlan P;
  if (!batch_plan_host(count, n_p, P)) return fail(-2, "every problem needs n >= 1");
  if (!factor_buf) return fail(-14, "factor buffer is NULL");
  if (factor_bytes < batch_factor_bytes(P, prec)) return fail(-15, "factor buffer too small");
  if (!sweep_rows_ok(opts)) return fail(-13, "sweep_rows must be 0, 64 or 128 (got %d)", opts->sweep_rows);
  const BatchWs W = batch_ws(P, count, N, S, prec, sweep_rows(opts));
  if (!ws) return fail(-16, "workspace is NULL");
  if (ws_bytes < W.total) return fail(-17, "workspace too small: %zu < %zu", ws_bytes, W.total);
  if (!d_out) return fail(-18, "output is NULL");
  if (!d_info) return fail(-19, "info is NULL");
  const uint64_t* lat = lattice_table(P.ldmax);
  if (!lat) return fail(-2, "could not build the lattice table");
  const mvn::BatchDesc* desc = (const mvn::BatchDesc*)d_plan;
  const int* order = (const int*)((const char*)d_plan + align_up(sizeof(mvn::BatchDesc) * (size_t)count));
  double* factor = (double*)factor_buf;
  void* low = prec == MVN_FP64 ? nullptr : (char*)factor_buf + align_up(sizeof(double) * (size_t)P.factor_elems);
  char* w = (char*)ws;
  double* at = (double*)(w + W.at);
  double* bt = (double*)(w + W.bt);
  uint64_t* dlat = (uint64_t*)(w + W.lat);
  double* ell = (double*)(w + W.ell);
  double* part = (double*)(w + W.part);
  int* bad = (int*)(w + W.bad);
  unsigned long long* counter = (unsigned long long*)(w + W.counter);
  hipError_t e = hipMemcpyAsync(dlat, lat, sizeof(uint64_t) * P.ldmax, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "lattice copy");
  e = mvn::launch_batch_build(desc, count, P.total_tiles, d_idx, d_locs, matern_of(kern), factor, d_info, stream);
  if (e != hipSuccess) return hip_fail(e, "batch build");
  e = mvn::launch_batch_cholesky(prec, desc, order, P.ld_rank.data(), count, factor, d_info, low,
                                 P.factor_elems, stream);
  if (e != hipSuccess) return hip_fail(e, "batch cholesky");
  e = mvn::launch_batch_setup(desc, count, P.nmax, d_a, d_b, d_mu, at, bt, bad, counter, stream);
  if (e != hipSuccess) return hip_fail(e, "batch setup");
  mvn::BatchSweepArgs a{};
  a.desc = desc;
  a.order = order;
  a.L = factor;
  a.Llow = prec == MVN_FP64 ? (const void*)factor : low;
  a.at = at;
  a.bt = bt;
  a.lattice = dlat;
  a.seed = seed;
  a.N = N;
  a.S = S;
  a.periodize = opts->periodize ? 1 : 0;
  a.prec = prec;
  a.yscr = (void*)(w + W.yscr);
  a.yslice = W.yslice;
  a.ell = ell;
  a.counter = counter;
  a.total_items = W.items;
  a.lplane = P.factor_elems;
  a.grid = W.grid;
  a.rows = sweep_rows(opts);
  e = batch_quad(prec, a.rows) ? mvn::launch_quad_batch_sweep(a, stream) : mvn::launch_batch_sweep(a, stream);
  if (e != hipSuccess) return hip_fail(e, "batch sweep");
  e = mvn::launch_batch_reduce(ell, count, N, S, part, d_info, bad, d_out, stream);
  if (e != hipSuccess) return hip_fail(e, "batch reduce");
  return 0;
}

}  // extern "C"
