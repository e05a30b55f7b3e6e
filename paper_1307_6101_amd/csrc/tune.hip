// Host side of the autotuner (declarations in tune.h).
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>

#include "tune.h"

namespace ddamg {

std::string tune_key(const Hierarchy& H, int nrhs) {
  hipDeviceProp_t prop;
  int dev = 0;
  DD_CHECK_HIP(hipGetDevice(&dev));
  DD_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  std::ostringstream k;
  const ddamg_params& p = H.p;
  k << arch << "|" << H.lv[0].dims[0] << "x" << H.lv[0].dims[1] << "x" << H.lv[0].dims[2] << "x" << H.lv[0].dims[3]
    << "|" << (p.precond_prec == DDAMG_F64 ? "f64" : (p.half_storage ? "f16" : "f32")) << "|L" << p.levels;
  for (int l = 0; l < p.levels - 1; ++l)
    k << "|a" << p.agg[l][0] << "." << p.agg[l][1] << "." << p.agg[l][2] << "." << p.agg[l][3] << "n" << p.ntv[l];
  k << "|" << (p.cycle == DDAMG_VCYCLE ? "V" : p.cycle == DDAMG_WCYCLE ? "W" : "K") << (p.graph ? "g" : "") << "|nrhs" << nrhs;
  return k.str();
}

std::vector<std::array<int, 4>> sap_candidates(const Hierarchy& H, int l) {
  std::vector<std::array<int, 4>> out;
  const int* e = H.lv[l].dims;
  for (int bs = 1; bs <= 8; ++bs) {
    bool ok = true;
    for (int mu = 0; mu < 3; ++mu) ok = ok && e[mu] % bs == 0 && (e[mu] / bs) % 2 == 0;
    if (!ok) continue;
    for (int bt = 1; bt <= 8; ++bt) {
      if (e[3] % bt != 0 || (e[3] / bt) % 2 != 0) continue;
      const int vol = bs * bs * bs * bt;
      if (vol < 8 || vol > 512) continue;
      out.push_back({bs, bs, bs, bt});
    }
  }
  return out;
}

namespace {

// one entry per line: "key": {"sap_block_l": [a, ..., l], "batch": n, "seconds": s}
bool parse_line(const std::string& line, std::string& key, TuneChoice& c) {
  const size_t q0 = line.find('"');
  const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
  if (q1 == std::string::npos) return false;
  key = line.substr(q0 + 1, q1 - q0 - 1);
  const size_t a = line.find('[', q1);
  if (a == std::string::npos) return false;
  int v[12];
  int batch = 0;
  double secs = 0;
  const int got = std::sscanf(line.c_str() + a,
                              "[%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d], \"batch\": %d, \"seconds\": %lf",
                              &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &v[10], &v[11],
                              &batch, &secs);
  if (got != 14) return false;
  for (int i = 0; i < 12; ++i) c.sap[i / 4][i % 4] = v[i];
  c.batch = batch;
  c.seconds = secs;
  return true;
}

std::map<std::string, TuneChoice> read_cache(const std::string& path) {
  std::map<std::string, TuneChoice> m;
  std::ifstream f(path);
  std::string line, key;
  while (std::getline(f, line)) {
    TuneChoice c;
    if (parse_line(line, key, c)) m[key] = c;
  }
  return m;
}

}  // namespace

bool tune_cache_lookup(const std::string& path, const std::string& key, TuneChoice& c) {
  const auto m = read_cache(path);
  const auto it = m.find(key);
  if (it == m.end()) return false;
  c = it->second;
  return true;
}

void tune_cache_store(const std::string& path, const std::string& key, const TuneChoice& c) {
  auto m = read_cache(path);
  m[key] = c;
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    DD_REQUIRE(f.good(), "cannot write the tuning cache " + tmp);
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      const TuneChoice& e = kv.second;
      f << "\"" << kv.first << "\": {\"sap_block_l\": [";
      for (int k = 0; k < 12; ++k) f << (k ? ", " : "") << e.sap[k / 4][k % 4];
      char tail[96];
      std::snprintf(tail, sizeof(tail), "], \"batch\": %d, \"seconds\": %.6g}", e.batch, e.seconds);
      f << tail << (++i < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  DD_REQUIRE(std::rename(tmp.c_str(), path.c_str()) == 0, "cannot replace the tuning cache " + path);
}

}  // namespace ddamg
