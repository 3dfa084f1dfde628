// Prints the TLR sweep's index tables (tlr_tables.h) for ranks read from
// stdin: "nt rs" then nt (nt - 1) / 2 ranks.  One table per line.
#include <stdio.h>

#include <vector>

#include "../../paper_2405_14892_amd/csrc/tlr_tables.h"

template <class V>
static void row(const char* name, const V& v) {
  printf("%s", name);
  for (const auto& x : v) printf(" %ld", (long)x);
  printf("\n");
}

int main() {
  int nt = 0, rs = 0;
  if (scanf("%d %d", &nt, &rs) != 2) return 1;
  std::vector<int> r(nt * (nt - 1) / 2 > 0 ? nt * (nt - 1) / 2 : 1, 0);
  for (int p = 0; p < nt * (nt - 1) / 2; ++p)
    if (scanf("%d", &r[p]) != 1) return 1;
  const mvn::TlrTables T = mvn::build_tlr_tables(nt, rs, r.data());
  printf("ksum %ld\n", T.ksum);
  row("k", T.k);
  row("zcol", T.zcol);
  row("kpad0", T.kpad0);
  row("kval", T.kval);
  row("vrow0", T.vrow0);
  row("ucol0", T.ucol0);
  row("zdst", T.zdst);
  return 0;
}
