// Host-side driver for the sanitizer test (built with g++ -fsanitize=
// address,undefined together with the library's host table code): runs the
// mesh builder, the batching and every reference/fragment/split table
// builder on a mesh read from a file, writes the mesh arrays it built for
// comparison with the library, and checks the mesh builder's error paths.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_2408_06698_amd/csrc/host_tables.hpp"

using namespace hopu;

static double sum(const std::vector<double>& v) {
  double s = 0;
  for (double x : v) s += x;
  return s;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: host_check <mesh.bin> <out.bin> <kmax>\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hdr[2];
  if (std::fread(hdr, 8, 2, f) != 2) return 2;
  const int dim = (int)hdr[0];
  const int64_t E = hdr[1];
  std::vector<int64_t> vid(E * (dim + 1));
  std::vector<double> xyz(E * (dim + 1) * dim);
  if (std::fread(vid.data(), 8, vid.size(), f) != vid.size() || std::fread(xyz.data(), 8, xyz.size(), f) != xyz.size())
    return 2;
  std::fclose(f);
  MeshData m;
  std::string err;
  if (!build_mesh(dim, E, vid.data(), xyz.data(), m, err)) {
    std::fprintf(stderr, "mesh rejected: %s\n", err.c_str());
    return 3;
  }
  Batches b;
  make_batches(m, b);
  FILE* o = std::fopen(argv[2], "wb");
  if (!o) return 2;
  const int64_t sizes[4] = {(int64_t)m.fid.size(), (int64_t)m.nbr.size(), (int64_t)m.geo.size(), (int64_t)b.elem.size()};
  std::fwrite(sizes, 8, 4, o);
  std::fwrite(m.fid.data(), 4, m.fid.size(), o);
  std::fwrite(m.nbr.data(), 4, m.nbr.size(), o);
  std::fwrite(m.geo.data(), 8, m.geo.size(), o);
  std::fwrite(b.elem.data(), 4, b.elem.size(), o);
  std::fclose(o);
  const int kmax = std::atoi(argv[3]);
  for (int k = 1; k <= kmax; ++k) {
    RefTables t;
    if (!make_ref_tables(dim, k, t, err)) {
      std::fprintf(stderr, "tables k=%d: %s\n", k, err.c_str());
      return 4;
    }
    FragTables f64, f32;
    make_frag_tables(t, ROWMAP_F64, f64);
    make_frag_tables(t, ROWMAP_F32, f32);
    BfTables b2, b3;
    make_bf16_tables(f32, t.sz, 2, b2);
    make_bf16_tables(f32, t.sz, 3, b3);
    std::printf("k=%d V %.17g mass_in %.17g psi_n %.17g vol_dV %.17g bf16 %zu\n", k, sum(t.V), sum(f64.mass_in),
                sum(f32.psi_n), sum(f64.vol_dV), b3.vol_VT.size());
  }
  // error paths of the mesh builder: a repeated vertex, a degenerate
  // element, a facet shared by three elements
  {
    std::vector<int64_t> v2 = vid;
    v2[1] = v2[0];
    MeshData bad;
    if (build_mesh(dim, E, v2.data(), xyz.data(), bad, err)) return 5;
    std::vector<double> x2 = xyz;
    for (int a = 0; a < dim; ++a) x2[dim + a] = x2[a];
    if (build_mesh(dim, E, vid.data(), x2.data(), bad, err)) return 5;
  }
  std::printf("ok\n");
  return 0;
}
