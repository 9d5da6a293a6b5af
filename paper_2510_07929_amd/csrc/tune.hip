// Persisted launch shapes.  Every shape an autotuner picks (or a kqr_set_*
// call installs) is recorded here; kqr_tune_save writes them to a JSON file
// keyed by the device architecture, kqr_tune_load (or KQR_TUNE_FILE at the
// first call that touches the device) installs the entries recorded for the
// current architecture, so a process starts with tuned shapes instead of
// sweeping again.
//
// File format (one entry per line, written and read only by this file):
//   {"arch": "gfx950:sramecc+:xnack-", "entries": [
//   {"kind": "apply", "k_dtype": 0, "mode": 0, "n": 50000, "m": 1, "a": 4, "b": 2, "c": 4, "wgs": 0, "us": 1440.1},
//   ...]}
// with (a, b, c) = apply: (rows, unroll, segments); kv: (nld, prefetch,
// segments); packed: (map, strip, -); otf: (strip, -, -) plus wgs.
#include "kernel_entry.h"
#include "kmulti.h"
#include "kqr_internal.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace kqr {

namespace {
std::mutex g_tune_mu;
// key: (kind, k_dtype, mode, size key) -> entry; later records replace earlier ones
std::map<std::tuple<std::string, int, int, int64_t>, TuneEntry> g_tune;

std::string device_arch() {
  int dev = 0;
  KQR_CHECK_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  KQR_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
  return std::string(prop.gcnArchName);
}

int64_t size_key(const TuneEntry& e) {
  // the size classes of each table: apply 0 / 8192 / 65536; kv powers of two
  // from 4096; otf tile rows 64 / 256 / 1024; packed has one class
  if (e.kind == "packed") return 0;
  if (e.kind == "apply") return e.n < 8192 ? 0 : (e.n < 65536 ? 1 : 2);
  if (e.kind == "kv") {
    int b = 0;
    while (b + 1 < 8 && (int64_t(4096) << b) < e.n) ++b;
    return b;
  }
  const int64_t nt = (e.n + kPkT - 1) / kPkT;
  return nt >= 1024 ? 3 : (nt >= 256 ? 2 : (nt >= 64 ? 1 : 0));
}

void install(const TuneEntry& e) {
  if (e.kind == "apply") {
    ApplyShape s;
    s.rows = e.a;
    s.unroll = e.b;
    s.segs = e.c;
    if (!apply_shape_supported(s)) fail(KQR_EINVAL, "tuning entry: unsupported apply shape");
    set_apply_shape(e.k_dtype, e.mode, e.n, s);
  } else if (e.kind == "kv") {
    KvShape s;
    s.nld = e.a;
    s.prefetch = e.b;
    s.segs = e.c;
    if (!kv_shape_supported(s)) fail(KQR_EINVAL, "tuning entry: unsupported K V shape");
    set_kv_shape(e.k_dtype, e.n, s);
  } else if (e.kind == "packed") {
    const PackedShape s{e.a, e.b};
    if (!packed_shape_supported(s)) fail(KQR_EINVAL, "tuning entry: unsupported packed shape");
    set_packed_shape(e.k_dtype, e.mode, s);
  } else if (e.kind == "otf") {
    if (e.a < 0 || e.a > kPkMaxStrip) fail(KQR_EINVAL, "tuning entry: unsupported on-the-fly strip");
    if (e.wgs != 0 && (e.wgs < 256 || e.wgs > (int64_t(1) << 20))) fail(KQR_EINVAL, "tuning entry: bad wgs");
    set_otf_strip_for(e.n, e.a);
    if (e.wgs > 0) set_otf_wgs(e.wgs);
  } else {
    fail(KQR_EINVAL, "tuning entry of unknown kind '%s'", e.kind.c_str());
  }
}

// value of "key": in line (number or quoted string); false if absent
bool field(const std::string& line, const char* key, std::string& out) {
  const std::string k = std::string("\"") + key + "\":";
  size_t pos = line.find(k);
  if (pos == std::string::npos) return false;
  pos += k.size();
  while (pos < line.size() && line[pos] == ' ') ++pos;
  if (pos < line.size() && line[pos] == '"') {
    const size_t e = line.find('"', pos + 1);
    if (e == std::string::npos) return false;
    out = line.substr(pos + 1, e - pos - 1);
    return true;
  }
  size_t e = pos;
  while (e < line.size() && line[e] != ',' && line[e] != '}') ++e;
  out = line.substr(pos, e - pos);
  return !out.empty();
}

int64_t num_field(const std::string& line, const char* key) {
  std::string v;
  if (!field(line, key, v)) fail(KQR_EINVAL, "tuning entry without \"%s\"", key);
  char* end = nullptr;
  const long long x = std::strtoll(v.c_str(), &end, 10);
  if (end == v.c_str()) fail(KQR_EINVAL, "tuning entry: \"%s\" is not a number", key);
  return int64_t(x);
}

std::once_flag g_autoload_once;
}  // namespace

void tune_record(const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[std::make_tuple(e.kind, e.k_dtype, e.mode, size_key(e))] = e;
}

int tune_save(const char* path) {
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) fail(KQR_EINVAL, "cannot write %s", path);
  std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", arch.c_str());
  size_t i = 0;
  for (const auto& kv : g_tune) {
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 "{\"kind\": \"%s\", \"k_dtype\": %d, \"mode\": %d, \"n\": %lld, \"m\": %d, \"a\": %d, \"b\": %d, "
                 "\"c\": %d, \"wgs\": %lld, \"us\": %.2f}%s\n",
                 e.kind.c_str(), e.k_dtype, e.mode, (long long)e.n, e.m, e.a, e.b, e.c, (long long)e.wgs, e.us,
                 ++i < g_tune.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok) fail(KQR_EHIP, "writing %s failed", path);
  return int(g_tune.size());
}

int tune_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) fail(KQR_EINVAL, "cannot read %s", path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  // the whole file is checked before anything is installed
  std::string file_arch;
  if (!field(text.substr(0, text.find('\n')), "arch", file_arch)) fail(KQR_EINVAL, "%s has no \"arch\"", path);
  std::vector<TuneEntry> entries;
  size_t pos = text.find('\n');
  while (pos != std::string::npos && pos + 1 < text.size()) {
    const size_t next = text.find('\n', pos + 1);
    const std::string line = text.substr(pos + 1, next == std::string::npos ? std::string::npos : next - pos - 1);
    pos = next;
    std::string kind;
    if (!field(line, "kind", kind)) continue;
    TuneEntry e;
    e.kind = kind;
    e.k_dtype = int(num_field(line, "k_dtype"));
    e.mode = int(num_field(line, "mode"));
    e.n = num_field(line, "n");
    e.m = int(num_field(line, "m"));
    e.a = int(num_field(line, "a"));
    e.b = int(num_field(line, "b"));
    e.c = int(num_field(line, "c"));
    e.wgs = num_field(line, "wgs");
    std::string us;
    if (field(line, "us", us)) e.us = std::atof(us.c_str());
    if ((e.k_dtype != KQR_FP32 && e.k_dtype != KQR_BF16) || e.mode < 0 || e.mode > 1)
      fail(KQR_EINVAL, "tuning entry: bad k_dtype or mode");
    entries.push_back(e);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    fail(KQR_ENODEVICE, "no HIP device available");
  }
  if (file_arch != device_arch()) return 0;  // tuned on another architecture: nothing applies
  for (const TuneEntry& e : entries) {
    install(e);
    tune_record(e);
  }
  return int(entries.size());
}

void tune_autoload() {
  std::call_once(g_autoload_once, [] {
    const char* path = std::getenv("KQR_TUNE_FILE");
    if (!path || !*path) return;
    try {
      tune_load(path);
    } catch (const Error& e) {
      std::fprintf(stderr, "[kqr] KQR_TUNE_FILE=%s not loaded: %s\n", path, e.what());
    }
  });
}

}  // namespace kqr
