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
//
// With --sapprox EPS the single record runs through dpc_sapprox_run with that eps,
// and the output ends with the n picked flags (uint8).
//
// With --decision the input is int64 n, int32 rho_min, int32 k, double d_cut, int32
// n_rho_bins, int32 n_delta_bins, then rho[n] (int32), delta[n], rho_edges and
// delta_edges (doubles); the output is int32 statuses of dpc_decision_top,
// dpc_decision_suggest and dpc_decision_histogram, int64 count, ids[k], deltas[k],
// rhos[k], double delta_min, int64 centers, int64 counts[bins].
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

int run_decision(const char *inp, const char *outp) {
  FILE *in = std::fopen(inp, "rb");
  if (!in) return 2;
  int64_t n;
  int32_t rho_min, k, nr, nd;
  double d_cut;
  if (std::fread(&n, 8, 1, in) != 1 || std::fread(&rho_min, 4, 1, in) != 1 || std::fread(&k, 4, 1, in) != 1 ||
      std::fread(&d_cut, 8, 1, in) != 1 || std::fread(&nr, 4, 1, in) != 1 || std::fread(&nd, 4, 1, in) != 1)
    return 2;
  std::vector<int32_t> rho(n);
  std::vector<double> delta(n), re(nr + 1), de(nd + 1);
  if (std::fread(rho.data(), 4, n, in) != size_t(n) || std::fread(delta.data(), 8, n, in) != size_t(n) ||
      std::fread(re.data(), 8, nr + 1, in) != size_t(nr + 1) || std::fread(de.data(), 8, nd + 1, in) != size_t(nd + 1))
    return 2;
  std::fclose(in);
  void *ws = std::aligned_alloc(256, DPC_DECISION_WS_BYTES);
  std::vector<int32_t> ids(k, -7), rhos(k, -7);
  std::vector<double> deltas(k, -7.0);
  std::vector<int64_t> counts(size_t(nr) * nd, -7);
  int64_t count = -7, centers = -7;
  double dmin = -7.0;
  const int32_t s1 = dpc_decision_top(n, rho.data(), delta.data(), rho_min, k, ids.data(), deltas.data(),
                                      rhos.data(), &count, ws, DPC_DECISION_WS_BYTES, nullptr);
  const int32_t s2 = dpc_decision_suggest(deltas.data(), &count, d_cut, &dmin, &centers, nullptr);
  const int32_t s3 = dpc_decision_histogram(n, rho.data(), delta.data(), re.data(), nr, de.data(), nd,
                                            counts.data(), nullptr);
  std::free(ws);
  FILE *out = std::fopen(outp, "wb");
  std::fwrite(&s1, 4, 1, out);
  std::fwrite(&s2, 4, 1, out);
  std::fwrite(&s3, 4, 1, out);
  std::fwrite(&count, 8, 1, out);
  std::fwrite(ids.data(), 4, k, out);
  std::fwrite(deltas.data(), 8, k, out);
  std::fwrite(rhos.data(), 4, k, out);
  std::fwrite(&dmin, 8, 1, out);
  std::fwrite(&centers, 8, 1, out);
  std::fwrite(counts.data(), 8, counts.size(), out);
  std::fclose(out);
  return 0;
}

int main(int argc, char **argv) {
  if (argc == 4 && std::string(argv[1]) == "--decision") return run_decision(argv[2], argv[3]);
  bool approx_mode = false, sapprox_mode = false;
  double eps = 0.0;
  if (argc == 4 && std::string(argv[1]) == "--approx") {
    approx_mode = true;
    argv[1] = argv[2];
    argv[2] = argv[3];
    argc = 3;
  } else if (argc == 5 && std::string(argv[1]) == "--sapprox") {
    sapprox_mode = true;
    eps = std::atof(argv[2]);
    argv[1] = argv[3];
    argv[2] = argv[4];
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
  const size_t wsb = approx_mode    ? dpc_approx_workspace_bytes(n, d, d_cut)
                     : sapprox_mode ? dpc_sapprox_workspace_bytes(n, d, d_cut, eps)
                                    : dpc_workspace_bytes(n, d, d_cut);
  void *ws = std::aligned_alloc(256, (wsb + 255) / 256 * 256);
  std::vector<int32_t> rho(n), dep(n), label(n);
  std::vector<double> delta(n);
  std::vector<uint8_t> approx(n, 2);
  int64_t ncenters = -1;
  const int32_t st =
      approx_mode    ? dpc_approx_run(pts.data(), n, d, d_cut, rho_min, delta_min, rho.data(), dep.data(),
                                      delta.data(), label.data(), &ncenters, approx.data(), ws, wsb, nullptr)
      : sapprox_mode ? dpc_sapprox_run(pts.data(), n, d, d_cut, eps, rho_min, delta_min, rho.data(), dep.data(),
                                       delta.data(), label.data(), &ncenters, approx.data(), ws, wsb, nullptr)
                     : dpc_run(pts.data(), n, d, d_cut, rho_min, delta_min, rho.data(), dep.data(), delta.data(),
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
  if (approx_mode || sapprox_mode) std::fwrite(approx.data(), 1, n, out);
  std::fclose(out);
  return 0;
}
