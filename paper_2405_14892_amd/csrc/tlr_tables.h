// Index tables of the tile low-rank SOV sweep (arXiv 2405.14892, Section
// III-E: the limit update of tile-row i through the low-rank tiles,
// sum_{j<i} U_ij (V'_ij^T Y_j)).  Plain C++: built on the host from the
// ranks of a factor, copied to the device once per probability call.
//
// Two products per 64-sample chunk use them:
//   * the Z product of tile column j, right after the samples y of tile j
//     are known: one GEMM over the V' rows of every tile (i, j), i > j,
//     stacked in order of i (M = sum_i k_ij rows, K = m), reading y of
//     tile j once for all of them;
//   * the update of tile-row i: one GEMM [U_i0 ... U_i,i-1] [Z_i0; ...] with
//     the ranks packed along K (K_i = sum_j k_ij, padded to a multiple of 16
//     with zero columns of U).
// Pair p = (i, j), i > j, has index i (i - 1) / 2 + j (the factor's order).
#pragma once
#include <stdint.h>

#include <vector>

namespace mvn {

struct TlrTables {
  int nt = 0;
  long ksum = 0;                // sum of the ranks
  std::vector<int> k;           // per pair: rank used (|rank| clipped to [0, rs])
  std::vector<long> zcol;       // nt + 1: first stacked V' row of tile column j
  std::vector<long> kpad0;      // nt + 1: first packed K index of tile-row i
  std::vector<int> kval;        // nt: K_i (unpadded)
  std::vector<long> vrow0;      // per pair: stacked V' row of its first row
  std::vector<long> ucol0;      // per pair: packed K index (within tile-row i) of its first column
  std::vector<long> zdst;       // ksum: Z row (packed, tile-row order) of stacked V' row
};

inline int pair_index(int i, int j) { return i * (i - 1) / 2 + j; }

// ranks: nt (nt - 1) / 2 entries, negative for a tile that reached the rank
// cap (its magnitude is the rank).
inline TlrTables build_tlr_tables(int nt, int rs, const int* ranks) {
  TlrTables T;
  T.nt = nt;
  const int np = nt * (nt - 1) / 2;
  T.k.assign(np, 0);
  for (int p = 0; p < np; ++p) {
    const long r = ranks[p] < 0 ? -(long)ranks[p] : (long)ranks[p];  // widened: -INT_MIN
    T.k[p] = (int)(r > rs ? rs : r);
  }
  T.zcol.assign(nt + 1, 0);
  T.vrow0.assign(np, 0);
  for (int j = 0; j < nt; ++j) {
    long row = T.zcol[j];
    for (int i = j + 1; i < nt; ++i) {
      const int p = pair_index(i, j);
      T.vrow0[p] = row;
      row += T.k[p];
    }
    T.zcol[j + 1] = row;
  }
  T.ksum = T.zcol[nt];
  T.kpad0.assign(nt + 1, 0);
  T.kval.assign(nt, 0);
  T.ucol0.assign(np, 0);
  for (int i = 0; i < nt; ++i) {
    long c = 0;
    for (int j = 0; j < i; ++j) {
      const int p = pair_index(i, j);
      T.ucol0[p] = c;
      c += T.k[p];
    }
    T.kval[i] = (int)c;
    T.kpad0[i + 1] = T.kpad0[i] + (c + 15) / 16 * 16;
  }
  T.zdst.assign(T.ksum, 0);
  for (int i = 1; i < nt; ++i)
    for (int j = 0; j < i; ++j) {
      const int p = pair_index(i, j);
      for (int q = 0; q < T.k[p]; ++q) T.zdst[T.vrow0[p] + q] = T.kpad0[i] + T.ucol0[p] + q;
    }
  return T;
}

}  // namespace mvn
