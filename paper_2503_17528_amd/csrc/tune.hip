// Tuning table of the library: decisions keyed by (device architecture, op,
// b, a, knob).  Sources, in order of precedence: internal overrides (the
// measurement hooks), environment variables (BTA_FACTOR_LOOKAHEAD,
// BTA_FACTOR_CACHED), the table (entries measured by the autotuners: the
// Python factor tuner and the first-use tuner of the batched selected
// inversion, and entries loaded from the JSON file named by BTA_TUNE_CACHE),
// then the built-in defaults.  The table is written back to BTA_TUNE_CACHE
// when a measurement adds an entry.  File format:
//   {"entries": {"gfx950|factor|b=2048|a=8|look": 8, ...}}
#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "bta_internal.hpp"
#include "bta_testing.h"

namespace bta {
namespace {

std::mutex g_tmu;
bool g_loaded = false;
std::map<std::string, long long> g_table;

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::string s(prop.gcnArchName);
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
  }
  return "gfx950";  // host-only use (no device): the only supported target
}

// {"entries": {"key": int, ...}} -> table (keys never contain quotes).
int parse_json(const std::string& txt, std::map<std::string, long long>& out) {
  const size_t e = txt.find("\"entries\"");
  if (e == std::string::npos) return 1;
  size_t i = txt.find('{', e);
  if (i == std::string::npos) return 2;
  ++i;
  for (;;) {
    while (i < txt.size() && (std::isspace((unsigned char)txt[i]) || txt[i] == ',')) ++i;
    if (i >= txt.size()) return 3;
    if (txt[i] == '}') return 0;
    if (txt[i] != '"') return 4;
    const size_t k1 = txt.find('"', i + 1);
    if (k1 == std::string::npos) return 5;
    const std::string key = txt.substr(i + 1, k1 - i - 1);
    i = txt.find(':', k1);
    if (i == std::string::npos) return 6;
    ++i;
    while (i < txt.size() && std::isspace((unsigned char)txt[i])) ++i;
    char* end = nullptr;
    const long long v = std::strtoll(txt.c_str() + i, &end, 10);
    if (end == txt.c_str() + i) return 7;
    out[key] = v;
    i = end - txt.c_str();
  }
}

int load_file(const char* path) {
  std::ifstream f(path);
  if (!f) return 1;
  std::stringstream ss;
  ss << f.rdbuf();
  std::map<std::string, long long> m;
  if (parse_json(ss.str(), m) != 0) return 2;
  for (auto& kv : m) g_table[kv.first] = kv.second;
  return 0;
}

int save_file(const char* path) {
  std::string s = "{\"entries\": {";
  bool first = true;
  for (auto& kv : g_table) {
    s += first ? "\n  " : ",\n  ";
    first = false;
    s += "\"" + kv.first + "\": " + std::to_string(kv.second);
  }
  s += "\n}}\n";
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return 1;
  const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
  if (std::fclose(f) != 0 || !ok) return 2;
  return std::rename(tmp.c_str(), path) == 0 ? 0 : 3;
}

void ensure_loaded() {
  if (g_loaded) return;
  g_loaded = true;
  if (const char* p = std::getenv("BTA_TUNE_CACHE")) (void)load_file(p);
}

}  // namespace

std::string tune_key(const char* op, int64_t b, int64_t a, const char* knob) {
  return device_arch() + "|" + op + "|b=" + std::to_string(b) + "|a=" + std::to_string(a) + "|" + knob;
}

bool tune_get(const std::string& key, long long* out) {
  std::lock_guard<std::mutex> lk(g_tmu);
  ensure_loaded();
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *out = it->second;
  return true;
}

void tune_set(const std::string& key, long long val, bool persist) {
  std::lock_guard<std::mutex> lk(g_tmu);
  ensure_loaded();
  g_table[key] = val;
  if (persist)
    if (const char* p = std::getenv("BTA_TUNE_CACHE")) (void)save_file(p);
}

bool env_int(const char* name, long long lo, long long hi, long long* out) {
  const char* s = std::getenv(name);
  if (!s || !*s) return false;
  char* end = nullptr;
  const long long v = std::strtoll(s, &end, 10);
  if (*end != 0 || v < lo || v > hi) return false;
  *out = v;
  return true;
}

}  // namespace bta

BTA_TESTING_API int bta_internal_tune_set(const char* key, long long value) {
  if (!key || !*key || std::strchr(key, '"')) return 1;
  bta::tune_set(key, value, false);
  return 0;
}

BTA_TESTING_API int bta_internal_tune_get(const char* key, long long* value) {
  if (!key || !value) return 1;
  return bta::tune_get(key, value) ? 0 : 2;
}

BTA_TESTING_API int bta_internal_tune_key(const char* op, int64_t b, int64_t a, const char* knob, char* out, int cap) {
  if (!op || !knob || !out || cap < 1) return 1;
  const std::string k = bta::tune_key(op, b, a, knob);
  if ((int)k.size() >= cap) return 2;
  std::memcpy(out, k.c_str(), k.size() + 1);
  return 0;
}

BTA_TESTING_API int bta_internal_tune_save(const char* path) {
  if (!path) return 1;
  std::lock_guard<std::mutex> lk(bta::g_tmu);
  bta::ensure_loaded();
  return bta::save_file(path);
}

BTA_TESTING_API int bta_internal_tune_load(const char* path) {
  if (!path) return 1;
  std::lock_guard<std::mutex> lk(bta::g_tmu);
  bta::ensure_loaded();
  return bta::load_file(path);
}

BTA_TESTING_API int bta_internal_tune_clear(void) {
  std::lock_guard<std::mutex> lk(bta::g_tmu);
  bta::g_loaded = true;
  bta::g_table.clear();
  return 0;
}

// Every table entry as "key=value" lines (up to cap bytes); returns the count.
BTA_TESTING_API int bta_internal_autotune_dump(char* out, int cap) {
  std::lock_guard<std::mutex> lk(bta::g_tmu);
  bta::ensure_loaded();
  std::string s;
  for (auto& kv : bta::g_table) s += kv.first + "=" + std::to_string(kv.second) + "\n";
  const int n = (int)std::min<size_t>(s.size(), cap > 0 ? (size_t)cap - 1 : 0);
  if (cap > 0) {
    std::memcpy(out, s.data(), n);
    out[n] = 0;
  }
  return (int)bta::g_table.size();
}
