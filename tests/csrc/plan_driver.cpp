// Host-only driver of the partition analysis for a sanitizer build: reads a
// mesh and a partition from a binary file (int64 n_vertices, int64 n_tets,
// float64 coords [n_vertices][3], int32 tets [n_tets][4], int32 partition
// [n_tets]), runs the analysis and the face-neighbour table, and prints the
// counts on one line.  Exit status 0 unless the file cannot be read.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "plan.hpp"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t nv = 0, nt = 0;
  if (std::fread(&nv, 8, 1, f) != 1 || std::fread(&nt, 8, 1, f) != 1 || nv < 0 || nt < 0) return 2;
  std::vector<double> coords(3 * nv);
  std::vector<int32_t> tets(4 * nt), part(nt);
  if (std::fread(coords.data(), 8, coords.size(), f) != coords.size() ||
      std::fread(tets.data(), 4, tets.size(), f) != tets.size() ||
      std::fread(part.data(), 4, part.size(), f) != part.size())
    return 2;
  std::fclose(f);
  ddfem::Plan P;
  std::string msg;
  int rc = ddfem::build_plan(nv, coords.data(), nt, tets.data(), part.data(), P, msg);
  if (rc != 0) {
    std::printf("rc %d %s\n", rc, msg.c_str());
    return 0;
  }
  std::vector<int32_t> nbr;
  int frc = ddfem::face_neighbors(P, nbr, msg);
  int64_t boundary = 0;
  for (int32_t x : nbr) boundary += x < 0;
  std::printf("rc 0 ne %lld nint %lld nsub %d nlam %lld ncorner %lld maxmult %d faces %d boundary %lld\n",
              (long long)P.ne, (long long)P.nint, P.nsub, (long long)P.nlambda(), (long long)P.ncorner(),
              P.max_mult, frc, (long long)boundary);
  return 0;
}
