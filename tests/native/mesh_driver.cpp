// Host-only driver of the mesh layer (mesh.cpp, q3.cpp), built by the CPU
// tests with AddressSanitizer and UndefinedBehaviorSanitizer.  Reads from stdin
//   base times n
//   n lines "level i j k"
// builds the mesh (refine + 2:1 balance + finalize) and prints, per level,
// the counts and the sorted node keys, node kinds, hanging rows and
// prolongation rows, so that the test can compare them with the oracle.
// argv[1]: "dirichlet" (default; also prints the local-smoothing levels),
// "noflux" (u . n = 0; also prints the fixed-component masks) or "q3" (the
// Q3-Q2 lattice levels).
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1907_06696_amd/csrc/mesh.h"

using namespace mfgmg;

int main(int argc, char** argv) {
  const std::string mode = argc > 1 ? argv[1] : "dirichlet";
  int base = 0, times = 0;
  long n = 0;
  if (std::scanf("%d %d %ld", &base, &times, &n) != 3) return 2;
  std::vector<int32_t> cells(size_t(4 * n));
  for (long i = 0; i < 4 * n; ++i)
    if (std::scanf("%d", &cells[size_t(i)]) != 1) return 2;
  Mesh m(base);
  if (mode == "noflux") m.set_noflux(true);
  if (mode == "q3") m.set_velocity_degree(3);
  if (n > 0) {
    std::string e = m.refine(cells.data(), n, times);
    if (!e.empty()) {
      std::printf("error %s\n", e.c_str());
      return 3;
    }
  }
  std::string e = m.finalize();
  if (!e.empty()) {
    std::printf("error %s\n", e.c_str());
    return 3;
  }
  std::printf("L %d\n", m.L());
  for (int ell = 1; ell <= m.L(); ++ell) {
    const Level& lv = mode == "q3" ? m.vlevel(ell) : m.level_transfer(ell);
    std::printf("level %d ncell %ld nnode %ld nhang %zu\n", ell, long(lv.ncell), long(lv.nnode), lv.hang.count());
    std::printf("keys");
    for (int64_t k : lv.key) std::printf(" %ld", long(k));
    std::printf("\ntypes");
    for (uint8_t t : lv.ntype) std::printf(" %d", int(t));
    std::printf("\nhang");
    for (size_t h = 0; h < lv.hang.count(); ++h)
      for (int64_t q = lv.hang.ptr[h]; q < lv.hang.ptr[h + 1]; ++q)
        std::printf(" %ld:%ld:%.15g", long(lv.hang.node[h]), long(lv.hang.master[size_t(q)]), lv.hang.weight[size_t(q)]);
    std::printf("\nprolong");
    if (ell >= 2)
      for (int64_t r = 0; r < lv.nnode; ++r)
        for (int64_t q = lv.P_ptr[size_t(r)]; q < lv.P_ptr[size_t(r + 1)]; ++q)
          std::printf(" %ld:%d:%.15g", long(r), lv.P_col[size_t(q)], lv.P_w[size_t(q)]);
    std::printf("\n");
    if (mode == "noflux") {
      std::printf("fix");
      for (uint8_t f : lv.fixmask) std::printf(" %d", int(f));
      std::printf("\n");
    }
  }
  const Level& lf = m.vleaf();
  std::printf("pressure npnode %ld nhang %zu\npkeys", long(lf.npnode), lf.phang.count());
  for (int64_t k : lf.pkey) std::printf(" %ld", long(k));
  std::printf("\n");
  if (mode != "dirichlet") return 0;
  // local-smoothing levels: cells, nodes, refinement-edge nodes, transfer entries, copied leaf nodes
  std::printf("local base %d", m.local_base());
  size_t copied = m.local_base_copy_leaf().size();
  for (int ell = m.local_base() + 1; ell <= m.L(); ++ell) {
    const LocalLevel& t = m.local_level(ell);
    long edge = 0;
    for (uint8_t k : t.kind) edge += k == 2;
    copied += t.copy_leaf.size();
    std::printf(" | %d %ld %ld %ld %zu", ell, long(t.mesh.ncell), long(t.mesh.nnode), edge, t.mesh.P_col.size());
  }
  std::printf(" | copied %zu\n", copied);
  return 0;
}
