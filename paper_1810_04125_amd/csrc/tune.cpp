// Launch-shape tunables and their table (hss_load_tunables): host only.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

#include "driver.h"

namespace hss {

namespace {

constexpr hss_tunables kDefaults = {2048, 32, 2048, kQrcpTarget};

struct Entry {
  std::string arch;
  int32_t family, precision;
  int64_t n_lo, n_hi;
  hss_tunables t;
};

std::mutex g_mu;
std::vector<Entry> g_table;
bool g_env_done = false;
thread_local const hss_tunables* g_active = nullptr;

bool valid(const hss_tunables& t) {
  return t.gemm_wg >= 64 && t.gemm_wg <= 65536 && t.gemm_max_split >= 1 && t.gemm_max_split <= 64 &&
         t.sample_wg >= 64 && t.sample_wg <= 65536 && t.qrcp_wg >= 64 && t.qrcp_wg <= HSS_QRCP_WG_MAX;
}

// Parses a table; throws HSS_ERR_INVALID_ARG naming the line.
std::vector<Entry> parse(const std::string& path) {
  std::ifstream f(path);
  if (!f) throw Error(HSS_ERR_INVALID_ARG, "cannot open tunables file " + path);
  std::vector<Entry> out;
  std::string line;
  int no = 0;
  while (std::getline(f, line)) {
    ++no;
    const size_t h = line.find('#');
    if (h != std::string::npos) line.resize(h);
    std::istringstream is(line);
    Entry e;
    if (!(is >> e.arch)) continue;   // blank
    if (!(is >> e.family >> e.precision >> e.n_lo >> e.n_hi >> e.t.gemm_wg >> e.t.gemm_max_split >> e.t.sample_wg >>
          e.t.qrcp_wg))
      throw Error(HSS_ERR_INVALID_ARG, path + ":" + std::to_string(no) + ": expected 9 fields");
    std::string extra;
    if (is >> extra) throw Error(HSS_ERR_INVALID_ARG, path + ":" + std::to_string(no) + ": extra field");
    if (!valid(e.t) || e.n_lo < 0 || e.n_hi <= e.n_lo)
      throw Error(HSS_ERR_INVALID_ARG, path + ":" + std::to_string(no) + ": value out of range");
    out.push_back(e);
  }
  return out;
}

void load_env_once() {   // g_mu held
  if (g_env_done) return;
  g_env_done = true;
  const char* p = std::getenv("HSS_TUNE_FILE");
  if (p && *p) g_table = parse(p);
}

hss_tunables lookup(const std::string& arch, int32_t family, int32_t precision, int64_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_env_once();
  for (const Entry& e : g_table)
    if (e.arch == arch && e.family == family && e.precision == precision && n >= e.n_lo && n < e.n_hi) return e.t;
  return kDefaults;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
    hipGetLastError();
    return "";
  }
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

}  // namespace

const hss_tunables& tune() { return g_active ? *g_active : kDefaults; }

TuneScope::TuneScope(const hss_tunables& t) : saved(g_active) { g_active = &t; }
TuneScope::~TuneScope() { g_active = saved; }

hss_tunables tunables_for(int32_t family, int32_t precision, int64_t n) {
  return lookup(device_arch(), family, precision, n);
}

}  // namespace hss

using namespace hss;

extern "C" {

hss_status hss_default_tunables(hss_tunables* out) {
  if (!out) return record_error(HSS_ERR_INVALID_ARG, "NULL argument");
  *out = kDefaults;
  return HSS_OK;
}

hss_status hss_load_tunables(const char* path) {
  try {
    std::vector<Entry> t;
    if (path && *path) t = parse(path);
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.swap(t);
    g_env_done = true;   // an explicit table replaces the environment's
    return HSS_OK;
  } catch (const Error& e) {
    return record_error(e.code, e.msg);
  }
}

hss_status hss_lookup_tunables(const char* arch, int32_t family, int32_t precision, int64_t n, hss_tunables* out) {
  if (!arch || !out) return record_error(HSS_ERR_INVALID_ARG, "NULL argument");
  try {
    *out = lookup(arch, family, precision, n);
    return HSS_OK;
  } catch (const Error& e) {
    return record_error(e.code, e.msg);
  }
}

}  // extern "C"
