// Host-only driver for the sanitizer build of the operator tables
// (op_build.cpp, Section 2.3 / Section 4.2 / Algorithm 4 tables).  Reads one
// system description from a text file, builds the host tables exactly as
// chfsi_op_build() does before its upload, and writes them as raw doubles /
// integers for comparison with the oracle.  Built with g++ and
// -fsanitize=address,undefined by tests/test_native_sanitize.py.
//
// Input (whitespace separated):  L ncell p natoms has_proj k0 k1 k2
// then per atom:                 x y z Z s w h_s h_p
// Output files in the output directory: x1d, cell_re, cell_im, dscale,
// vdiag, hcoef (float64), atom_ptr (int64), atom_node (int32), atom_val
// (float64; 4 or 8 values per entry), pair_ptr, pair_atom (int32), and
// "sizes" (text: M E mcell cplx npairs).
#include <cstdio>
#include <fstream>
#include <string>
#include <vector>

#include "../../paper_2203_07820_amd/csrc/internal.h"

template <typename T>
static bool dump(const std::string& path, const std::vector<T>& v) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) return false;
  const size_t n = v.empty() ? 0 : std::fwrite(v.data(), sizeof(T), v.size(), f);
  std::fclose(f);
  return n == v.size();
}

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s system.txt outdir\n", argv[0]);
    return 2;
  }
  std::ifstream in(argv[1]);
  chfsi_system sys{};
  in >> sys.L >> sys.ncell >> sys.p >> sys.natoms >> sys.has_proj >> sys.k[0] >> sys.k[1] >> sys.k[2];
  if (!in || sys.natoms < 0) return 2;
  std::vector<double> pos(3 * sys.natoms), Z(sys.natoms), s(sys.natoms), w(sys.natoms), hs(sys.natoms),
      hp(sys.natoms);
  for (int a = 0; a < sys.natoms; ++a)
    in >> pos[3 * a] >> pos[3 * a + 1] >> pos[3 * a + 2] >> Z[a] >> s[a] >> w[a] >> hs[a] >> hp[a];
  if (!in) return 2;
  sys.pos = pos.data();
  sys.Z = Z.data();
  sys.s = s.data();
  sys.w = w.data();
  sys.h_s = hs.data();
  sys.h_p = hp.data();
  chfsi::HostTables t;
  const std::string err = chfsi::build_tables(sys, t);
  if (!err.empty()) {
    std::fprintf(stderr, "build_tables: %s\n", err.c_str());
    return 1;
  }
  const std::string d = argv[2];
  bool ok = dump(d + "/x1d", t.x1d) && dump(d + "/cell_re", t.cell_re) && dump(d + "/cell_im", t.cell_im) &&
            dump(d + "/dscale", t.dscale) && dump(d + "/vdiag", t.vdiag) && dump(d + "/hcoef", t.hcoef) &&
            dump(d + "/atom_ptr", t.atom_ptr) && dump(d + "/atom_node", t.atom_node) &&
            dump(d + "/atom_val", t.atom_val) && dump(d + "/pair_ptr", t.pair_ptr) &&
            dump(d + "/pair_atom", t.pair_atom);
  std::ofstream sz(d + "/sizes");
  sz << t.M << " " << t.E << " " << t.mcell << " " << (t.cplx ? 1 : 0) << " " << t.pair_atom.size() << "\n";
  return ok && sz ? 0 : 1;
}
