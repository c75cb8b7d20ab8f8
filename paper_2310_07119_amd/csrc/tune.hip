// Tuning cache of the on-device autotuner (the measurement itself is
// tw_plan_autotune in api.hip).
//
// Two kernel organisations exist for passes along y and z (kernels_step.hip:
// pencils interleaved across wavefronts with workgroup-wide exchanges;
// kernels_cols.hip: coalesced LDS tiles with wavefront-local exchanges). Which
// is faster depends on precision, length and register pressure, so plans
// measure both and keep the faster. Results are cached in a small JSON object
//   {"<arch>|D<d>|<n0>x<n1>x<n2>|<precision>|pairs<p>": {"cols_variant": V, "us": [t0, t1]}, ...}
// at $TW_TUNE_CACHE, else $XDG_CACHE_HOME/twa_mi355x_tune.json, else
// $HOME/.cache/twa_mi355x_tune.json. A missing or unreadable cache only means
// the measurement runs again.
#include <sys/stat.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace tw {
namespace {

std::string cache_path() {
  if (const char* p = getenv("TW_TUNE_CACHE")) return p;
  if (const char* x = getenv("XDG_CACHE_HOME")) return std::string(x) + "/twa_mi355x_tune.json";
  if (const char* h = getenv("HOME")) return std::string(h) + "/.cache/twa_mi355x_tune.json";
  return "";
}

std::string read_file(const std::string& path) {
  std::string out;
  FILE* f = path.empty() ? nullptr : fopen(path.c_str(), "rb");
  if (!f) return out;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) out.append(buf, n);
  fclose(f);
  return out;
}

void make_parent_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

}  // namespace

std::string tune_key(const Plan& P) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, P.device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|D%d|%dx%dx%d|%s|pairs%lld%s", arch.c_str(), P.dim, P.n[0], P.n[1], P.n[2],
           P.fp32 ? "fp32" : "fp64", (long long)P.npairs, P.transpose2d ? "|alt" : "");
  return buf;
}

int tune_cache_lookup(const std::string& key) {
  const std::string text = read_file(cache_path());
  const size_t k = text.find("\"" + key + "\"");
  if (k == std::string::npos) return -1;
  const size_t v = text.find("\"cols_variant\":", k);
  if (v == std::string::npos) return -1;
  const int val = atoi(text.c_str() + v + 15);
  return (val == 0 || val == 1) ? val : -1;
}

void tune_cache_store(const std::string& key, int variant, const double us[2]) {
  const std::string path = cache_path();
  if (path.empty()) return;
  std::string text = read_file(path);
  if (text.find("\"" + key + "\"") != std::string::npos) return;  // first measurement wins
  char entry[512];
  snprintf(entry, sizeof(entry), "\"%s\": {\"cols_variant\": %d, \"us\": [%.1f, %.1f]}", key.c_str(), variant, us[0],
           us[1]);
  const size_t open = text.find('{');
  const size_t close = text.rfind('}');
  if (open == std::string::npos || close == std::string::npos || close < open) {
    text = std::string("{\n  ") + entry + "\n}\n";
  } else {
    const bool empty_obj = text.find('"', open) == std::string::npos;
    text = text.substr(0, close);
    while (!text.empty() && (text.back() == '\n' || text.back() == ' ')) text.pop_back();
    text += (empty_obj ? std::string("\n  ") : std::string(",\n  ")) + entry + "\n}\n";
  }
  make_parent_dirs(path);
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return;
  const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
  fclose(f);
  if (ok) (void)rename(tmp.c_str(), path.c_str());
}

}  // namespace tw
