// Host-only tool for test_label_tables.py: reads cell labels of a padded box
// (raw bytes, x fastest) and writes, for every multigrid level, the flag
// words and Vanka local inverses that csrc/host_tables.hpp builds, so the
// test can compare them with the oracle's masks, diagonals and local
// matrices.  Usage: label_tables_dump nx ny nz levels labels.bin out_prefix
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_2312_10615_amd/csrc/host_tables.hpp"

using namespace sg;

int main(int argc, char** argv) {
  if (argc != 7) return 2;
  const int nx = std::atoi(argv[1]), ny = std::atoi(argv[2]), nz = std::atoi(argv[3]), L = std::atoi(argv[4]);
  Labels lab;
  lab.nx = nx;
  lab.ny = ny;
  lab.nz = nz;
  lab.v.resize((size_t)(nx + 2) * (ny + 2) * (nz + 2));
  FILE* f = std::fopen(argv[5], "rb");
  if (!f || std::fread(lab.v.data(), 1, lab.v.size(), f) != lab.v.size()) return 3;
  std::fclose(f);
  const std::string out = argv[6];
  for (int l = 0; l < L; ++l) {
    if (l > 0) lab = coarsen(lab);
    const Geom g = make_geom(nx, ny, nz, 1.0 / nx, 1.0, 1e-3, l);
    LevelLabels t;
    if (!label_tables(g, lab, t)) return 4;
    // per padded cell (x fastest): the flag word of its slot
    std::vector<uint32_t> w((size_t)(g.nx + 2) * (g.ny + 2) * (g.nz + 2));
    for (int K = 0; K < g.nz + 2; ++K)
      for (int J = 0; J < g.ny + 2; ++J)
        for (int I = 0; I < g.nx + 2; ++I) w[lab.idx(I, J, K)] = t.flags[g.at(g.idx(I, J, K))];
    FILE* o = std::fopen((out + "_flags" + std::to_string(l) + ".bin").c_str(), "wb");
    std::fwrite(w.data(), 4, w.size(), o);
    std::fclose(o);
    o = std::fopen((out + "_kinv" + std::to_string(l) + ".bin").c_str(), "wb");
    std::fwrite(t.kinv.data(), 8, t.kinv.size(), o);
    std::fclose(o);
    o = std::fopen((out + "_labels" + std::to_string(l) + ".bin").c_str(), "wb");
    std::fwrite(lab.v.data(), 1, lab.v.size(), o);
    std::fclose(o);
  }
  return 0;
}
