// Tuning cache: the detection kernel chosen per shape class and the launch
// form chosen per batch shape mix, as measured by apsm_batch_tune, keyed by
// the GPU architecture name and the HIP runtime version so that a saved cache
// applies only where it was measured.  Host memory, one mutex; saved and
// loaded as a JSON object of string pairs.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "apsm_internal.h"

namespace apsm {
namespace {

std::mutex g_mutex;
std::map<std::string, std::string> g_cache;   // key -> choice
std::string g_device;                          // "<arch>|hip<version>", looked up once

// The current device's key prefix; "unknown" where no GPU answers.
const std::string& device_key() {
  if (!g_device.empty()) return g_device;
  int dev = 0, ver = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);     // drop feature suffixes
  } else {
    (void)hipGetLastError();
    return g_device = "unknown";
  }
  if (hipRuntimeGetVersion(&ver) != hipSuccess) ver = 0;
  g_device = arch + "|hip" + std::to_string(ver);
  return g_device;
}

std::string kernel_key(int M2, int K) {
  const int m2p = M2 <= 16 ? 16 : M2 <= 32 ? 32 : 64;
  return device_key() + "|detect|m2p" + std::to_string(m2p) + "|k" + std::to_string(K);
}

std::string form_key(uint64_t sig) {
  char buf[32];
  std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)sig);
  return device_key() + "|form|" + buf;
}

// JSON string body: the keys and values here hold no quotes or backslashes,
// but escape them anyway.
std::string quoted(const std::string& s) {
  std::string o = "\"";
  for (char c : s) {
    if (c == '"' || c == '\\') o += '\\';
    o += c;
  }
  return o + "\"";
}

}  // namespace

int detect_kernel_for(int M2, int K) {
  if (!detect_dual(M2, K)) return kDetectWide;
  std::lock_guard<std::mutex> lock(g_mutex);
  auto f = g_cache.find(kernel_key(M2, K));
  if (f == g_cache.end()) return detect_default_kernel(M2, K);
  return f->second == "f16" ? kDetectF16 : kDetectWide;
}

void tune_set_kernel(int M2, int K, int kernel) {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_cache[kernel_key(M2, K)] = kernel == kDetectF16 ? "f16" : "wide";
}

bool tune_get_form(uint64_t sig, bool* persistent) {
  std::lock_guard<std::mutex> lock(g_mutex);
  auto f = g_cache.find(form_key(sig));
  if (f == g_cache.end()) return false;
  *persistent = f->second == "persistent";
  return true;
}

void tune_set_form(uint64_t sig, bool persistent) {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_cache[form_key(sig)] = persistent ? "persistent" : "plain";
}

void tune_clear() {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_cache.clear();
}

}  // namespace apsm

extern "C" {

int apsm_tune_save(const char* path) {
  if (!path) return APSM_ERR_INVALID_ARG;
  std::string text = "{\n";
  {
    std::lock_guard<std::mutex> lock(apsm::g_mutex);
    size_t i = 0;
    for (const auto& kv : apsm::g_cache) {
      text += "  " + apsm::quoted(kv.first) + ": " + apsm::quoted(kv.second);
      text += ++i < apsm::g_cache.size() ? ",\n" : "\n";
    }
  }
  text += "}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return APSM_ERR_INVALID_ARG;
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  return (std::fclose(f) == 0 && ok) ? APSM_OK : APSM_ERR_INVALID_ARG;
}

int apsm_tune_load(const char* path) {
  if (!path) return APSM_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return APSM_ERR_INVALID_ARG;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  std::fclose(f);
  // a flat object of string pairs: "key": "value", ...
  std::map<std::string, std::string> parsed;
  size_t p = text.find('{');
  if (p == std::string::npos) return APSM_ERR_INVALID_ARG;
  auto skip = [&](size_t q) {
    while (q < text.size() && (text[q] == ' ' || text[q] == '\n' || text[q] == '\r' || text[q] == '\t')) ++q;
    return q;
  };
  auto string_at = [&](size_t& q, std::string& out) {
    q = skip(q);
    if (q >= text.size() || text[q] != '"') return false;
    out.clear();
    for (++q; q < text.size() && text[q] != '"'; ++q) {
      if (text[q] == '\\' && q + 1 < text.size()) ++q;
      out += text[q];
    }
    if (q >= text.size()) return false;
    ++q;
    return true;
  };
  p = skip(p + 1);
  while (p < text.size() && text[p] != '}') {
    std::string k, v;
    if (!string_at(p, k)) return APSM_ERR_INVALID_ARG;
    p = skip(p);
    if (p >= text.size() || text[p] != ':') return APSM_ERR_INVALID_ARG;
    if (!string_at(++p, v)) return APSM_ERR_INVALID_ARG;
    if (v != "f16" && v != "wide" && v != "persistent" && v != "plain") return APSM_ERR_INVALID_ARG;
    parsed[k] = v;
    p = skip(p);
    if (p < text.size() && text[p] == ',') p = skip(p + 1);
  }
  if (p >= text.size()) return APSM_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(apsm::g_mutex);
  for (const auto& kv : parsed) apsm::g_cache[kv.first] = kv.second;
  return APSM_OK;
}

void apsm_shutdown(void) { apsm::tune_clear(); }

}  // extern "C"
