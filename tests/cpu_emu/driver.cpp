// Runs dpc_run from the library's kernel sources built for the CPU (see
// hip/hip_runtime.h here).  Input file: int64 n, int32 d, double d_cut, int32
// rho_min, double delta_min, int32 points[n*d].  Output file: int32 status of
// dpc_run, int32 status of dpc_sync_status, int64 ncenters, then rho, dep,
// delta and label arrays.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dpc.h"

int main(int argc, char **argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE *in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t n;
  int32_t d, rho_min;
  double d_cut, delta_min;
  if (std::fread(&n, 8, 1, in) != 1 || std::fread(&d, 4, 1, in) != 1 || std::fread(&d_cut, 8, 1, in) != 1 ||
      std::fread(&rho_min, 4, 1, in) != 1 || std::fread(&delta_min, 8, 1, in) != 1)
    return 2;
  std::vector<int32_t> pts(size_t(n) * d);
  if (std::fread(pts.data(), 4, pts.size(), in) != pts.size()) return 2;
  std::fclose(in);
  const size_t wsb = dpc_workspace_bytes(n, d, d_cut);
  void *ws = std::aligned_alloc(256, (wsb + 255) / 256 * 256);
  std::vector<int32_t> rho(n), dep(n), label(n);
  std::vector<double> delta(n);
  int64_t ncenters = -1;
  const int32_t st = dpc_run(pts.data(), n, d, d_cut, rho_min, delta_min, rho.data(), dep.data(), delta.data(),
                             label.data(), &ncenters, ws, wsb, nullptr);
  const int32_t st2 = dpc_sync_status(ws, nullptr);
  std::free(ws);
  FILE *out = std::fopen(argv[2], "wb");
  std::fwrite(&st, 4, 1, out);
  std::fwrite(&st2, 4, 1, out);
  std::fwrite(&ncenters, 8, 1, out);
  std::fwrite(rho.data(), 4, n, out);
  std::fwrite(dep.data(), 4, n, out);
  std::fwrite(delta.data(), 8, n, out);
  std::fwrite(label.data(), 4, n, out);
  std::fclose(out);
  return 0;
}
