// Runs dpc_run from the library's kernel sources built for the CPU (see
// hip/hip_runtime.h here).  Input file: int64 n, int32 d, double d_cut, int32
// rho_min, double delta_min, int32 points[n*d].  Output file: int32 status of
// dpc_run, int32 status of dpc_sync_status, int64 ncenters, then rho, dep,
// delta and label arrays.
//
// With --batch the input holds int32 njobs and then njobs such records; all
// jobs run through dpc_batch_run and the output holds one record per job
// (the status fields are those of the batch calls).  --tuning SPEC (batch only)
// gives every job the plan options of SPEC, "key=value" items separated by ';':
// subdiv, strip, ring, gm, lanes, open, and stages=K:group,K:group,...
//
// With --approx the single record runs through dpc_approx_run instead, and the
// output ends with the n approx flags (uint8).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dpc.h"

struct Rec {
  int64_t n;
  int32_t d, rho_min;
  double d_cut, delta_min;
  std::vector<int32_t> pts, rho, dep, label;
  std::vector<double> delta;
  int64_t ncenters = -1;
};

bool read_rec(FILE *in, Rec &r) {
  if (std::fread(&r.n, 8, 1, in) != 1 || std::fread(&r.d, 4, 1, in) != 1 || std::fread(&r.d_cut, 8, 1, in) != 1 ||
      std::fread(&r.rho_min, 4, 1, in) != 1 || std::fread(&r.delta_min, 8, 1, in) != 1)
    return false;
  r.pts.resize(size_t(r.n) * r.d);
  if (std::fread(r.pts.data(), 4, r.pts.size(), in) != r.pts.size()) return false;
  r.rho.resize(r.n);
  r.dep.resize(r.n);
  r.label.resize(r.n);
  r.delta.resize(r.n);
  return true;
}

void write_rec(FILE *out, int32_t st, int32_t st2, const Rec &r) {
  std::fwrite(&st, 4, 1, out);
  std::fwrite(&st2, 4, 1, out);
  std::fwrite(&r.ncenters, 8, 1, out);
  std::fwrite(r.rho.data(), 4, r.n, out);
  std::fwrite(r.dep.data(), 4, r.n, out);
  std::fwrite(r.delta.data(), 8, r.n, out);
  std::fwrite(r.label.data(), 4, r.n, out);
}

// Plan options from a --tuning SPEC (see above); false on a malformed spec.
bool parse_tuning(const std::string &spec, dpc_tuning *t) {
  std::memset(t, 0, sizeof(*t));
  size_t at = 0;
  while (at < spec.size()) {
    size_t end = spec.find(';', at);
    if (end == std::string::npos) end = spec.size();
    const std::string item = spec.substr(at, end - at);
    at = end + 1;
    const size_t eq = item.find('=');
    if (eq == std::string::npos) return false;
    const std::string k = item.substr(0, eq), v = item.substr(eq + 1);
    if (k == "stages") {
      int n = 0;
      for (size_t c = 0; c < v.size() && n < 4;) {
        int K = 0, g = 1;
        if (std::sscanf(v.c_str() + c, "%d:%d", &K, &g) < 1) return false;
        t->stage_radius[n] = K;
        t->stage_group[n] = g;
        ++n;
        const size_t comma = v.find(',', c);
        if (comma == std::string::npos) break;
        c = comma + 1;
      }
      t->nstages = n;
      continue;
    }
    const int x = std::atoi(v.c_str());
    if (k == "subdiv") t->subdiv = x;
    else if (k == "strip") t->strip_cells = x;
    else if (k == "ring") t->ring_cap = x;
    else if (k == "gm") t->grid_dims = x;
    else if (k == "lanes") t->lanes = x;
    else if (k == "open") t->open_radius = x;
    else return false;
  }
  return true;
}

int run_batch(const char *inp, const char *outp, const dpc_tuning *tuning) {
  FILE *in = std::fopen(inp, "rb");
  if (!in) return 2;
  int32_t njobs = 0;
  if (std::fread(&njobs, 4, 1, in) != 1 || njobs < 1) return 2;
  std::vector<Rec> recs(njobs);
  for (auto &r : recs)
    if (!read_rec(in, r)) return 2;
  std::fclose(in);
  std::vector<dpc_job> jobs(njobs);
  for (int32_t i = 0; i < njobs; ++i) {
    Rec &r = recs[i];
    jobs[i] = dpc_job{r.pts.data(), r.n, r.d, r.d_cut, r.rho_min, r.delta_min, r.rho.data(), r.dep.data(),
                      r.delta.data(), r.label.data(), &r.ncenters};
  }
  dpc_batch *b = nullptr;
  size_t wsb = 0;
  std::vector<dpc_tuning> tun(njobs);
  if (tuning)
    for (auto &t : tun) t = *tuning;
  int32_t st = dpc_batch_plan(jobs.data(), njobs, tuning ? tun.data() : nullptr, &b, &wsb);
  int32_t st2 = st;
  if (st == DPC_OK) {
    void *ws = std::aligned_alloc(256, (wsb + 255) / 256 * 256);
    st = dpc_batch_bind(b, ws, wsb);
    if (st == DPC_OK) st = dpc_batch_run(b, ws, nullptr);
    int32_t bad = -1;
    st2 = dpc_batch_sync_status(b, ws, nullptr, &bad);
    std::free(ws);
    dpc_batch_free(b);
  }
  FILE *out = std::fopen(outp, "wb");
  for (auto &r : recs) write_rec(out, st, st2, r);
  std::fclose(out);
  return 0;
}

int main(int argc, char **argv) {
  bool approx_mode = false;
  if (argc == 4 && std::string(argv[1]) == "--approx") {
    approx_mode = true;
    argv[1] = argv[2];
    argv[2] = argv[3];
    argc = 3;
  }
  if (argc == 4 && std::string(argv[1]) == "--batch") return run_batch(argv[2], argv[3], nullptr);
  if (argc == 6 && std::string(argv[1]) == "--batch" && std::string(argv[2]) == "--tuning") {
    dpc_tuning t;
    if (!parse_tuning(argv[3], &t)) {
      std::fprintf(stderr, "bad --tuning spec\n");
      return 2;
    }
    return run_batch(argv[4], argv[5], &t);
  }
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s [--batch] input output\n", argv[0]);
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
  const size_t wsb = approx_mode ? dpc_approx_workspace_bytes(n, d, d_cut) : dpc_workspace_bytes(n, d, d_cut);
  void *ws = std::aligned_alloc(256, (wsb + 255) / 256 * 256);
  std::vector<int32_t> rho(n), dep(n), label(n);
  std::vector<double> delta(n);
  std::vector<uint8_t> approx(n, 2);
  int64_t ncenters = -1;
  const int32_t st = approx_mode
                         ? dpc_approx_run(pts.data(), n, d, d_cut, rho_min, delta_min, rho.data(), dep.data(),
                                          delta.data(), label.data(), &ncenters, approx.data(), ws, wsb, nullptr)
                         : dpc_run(pts.data(), n, d, d_cut, rho_min, delta_min, rho.data(), dep.data(),
                                   delta.data(), label.data(), &ncenters, ws, wsb, nullptr);
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
  if (approx_mode) std::fwrite(approx.data(), 1, n, out);
  std::fclose(out);
  return 0;
}
