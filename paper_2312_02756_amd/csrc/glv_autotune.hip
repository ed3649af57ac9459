// Host side of the jagged reduction's autotuner (declared in glv_autotune.h):
// dataset signatures, cache keys, and the JSON cache file.
#include "glv_autotune.h"

#include <stdio.h>

#include <algorithm>
#include <cerrno>
#include <cstring>
#include <map>
#include <mutex>

namespace glv {
namespace tune {

namespace {

std::mutex g_mu;
std::map<std::string, Tiling> g_by_key;

int size_class(int64_t n) {
  if (n <= 0) return 0;
  int b = 1;
  while (b < 40 && (n >> b) != 0) ++b;
  return b;  // 2^(b-1) <= n < 2^b
}

int log2_floor(int64_t n) {
  int e = 0;
  while (n > 1) {
    n >>= 1;
    ++e;
  }
  return e;
}

// Minimal reader of the cache file's JSON.
struct Reader {
  const std::string& s;
  size_t i = 0;
  std::string err;
  explicit Reader(const std::string& text) : s(text) {}
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  }
  bool lit(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool expect(char c) {
    if (lit(c)) return true;
    if (err.empty()) err = std::string("expected '") + c + "' at byte " + std::to_string(i);
    return false;
  }
  bool str(std::string* out) {
    if (!expect('"')) return false;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      const char c = s[i++];
      if (c == '\\' || (unsigned char)c < 0x20) {
        err = "unsupported character in a string at byte " + std::to_string(i - 1);
        return false;
      }
      out->push_back(c);
    }
    if (i >= s.size()) {
      err = "unterminated string";
      return false;
    }
    ++i;
    return true;
  }
  bool integer(long long* v) {
    ws();
    size_t j = i;
    if (j < s.size() && s[j] == '-') ++j;
    const size_t d0 = j;
    while (j < s.size() && s[j] >= '0' && s[j] <= '9') ++j;
    if (j == d0 || j - d0 > 9) {
      err = "expected an integer at byte " + std::to_string(i);
      return false;
    }
    *v = std::stoll(s.substr(i, j - i));
    i = j;
    return true;
  }
  bool field(const char* name) {
    std::string k;
    if (!str(&k)) return false;
    if (k != name) {
      err = std::string("expected field \"") + name + "\", found \"" + k + "\"";
      return false;
    }
    return expect(':');
  }
};

}  // namespace

std::string signature_of_sizes(int64_t n_events, const int64_t* sizes, int64_t n_sampled) {
  std::string sig = "e" + std::to_string(n_events > 0 ? log2_floor(n_events) : -1);
  if (n_sampled <= 0) return sig;
  std::vector<int64_t> hist(41, 0);
  for (int64_t k = 0; k < n_sampled; ++k) ++hist[size_class(sizes[k])];
  sig += ";";
  bool first = true;
  for (int b = 0; b < 41; ++b) {
    // share in 5 % steps, rounded to nearest
    const int64_t steps = (hist[b] * 20 + n_sampled / 2) / n_sampled;
    if (steps == 0) continue;
    if (!first) sig += ",";
    sig += std::to_string(b) + ":" + std::to_string(steps * 5);
    first = false;
  }
  return sig;
}

hipError_t signature(int64_t n_events, const int64_t* offsets, hipStream_t s, std::string* sig) {
  std::vector<int64_t> sizes;
  if (n_events > 0) {
    std::vector<std::pair<int64_t, int64_t>> runs;  // (first event, count)
    if (n_events <= kSampleEvents) {
      runs.push_back({0, n_events});
    } else {
      const int64_t len = kSampleEvents / kSampleRuns;
      for (int r = 0; r < kSampleRuns; ++r) runs.push_back({r * (n_events - len) / (kSampleRuns - 1), len});
    }
    std::vector<int64_t> buf;
    for (const auto& run : runs) {
      buf.resize((size_t)run.second + 1);
      hipError_t e = hipMemcpyAsync(buf.data(), offsets + run.first, buf.size() * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      for (int64_t k = 0; k < run.second; ++k) sizes.push_back(buf[k + 1] - buf[k]);
    }
  }
  *sig = signature_of_sizes(n_events, sizes.data(), (int64_t)sizes.size());
  return hipSuccess;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "none";
  }
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string make_key(glv_dtype dt, glv_coords co, const char* what, const std::string& sig) {
  static const char* coords[] = {"PxPyPzE", "PtEtaPhiM", "PtEtaPhiE", "PxPyPzM"};
  const char* c = ((int)co >= 0 && (int)co < 4) ? coords[(int)co] : "?";
  return arch_name() + "|" + (dt == GLV_F64 ? "f64" : "f32") + "|" + c + "|" + what + "|" + sig;
}

FileState load(const char* path, Entries* out, std::string* why) {
  out->clear();
  FILE* f = fopen(path, "rb");
  if (!f) {
    if (errno == ENOENT) return FileState::kMissing;
    *why = std::string("cannot open: ") + strerror(errno);
    return FileState::kCorrupt;
  }
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  const bool io_err = ferror(f) != 0;
  fclose(f);
  if (io_err) {
    *why = "read error";
    return FileState::kCorrupt;
  }
  Reader r(text);
  std::string fmt;
  bool ok = r.expect('{') && r.field("format") && r.str(&fmt);
  if (ok && fmt != "glv-autotune-1") {
    r.err = "unknown format \"" + fmt + "\"";
    ok = false;
  }
  ok = ok && r.expect(',') && r.field("entries") && r.expect('[');
  if (ok && !r.lit(']')) {
    do {
      std::string key;
      long long v[4];
      ok = r.expect('{') && r.field("key") && r.str(&key) && r.expect(',') && r.field("tiling") && r.expect('[') &&
           r.integer(&v[0]) && r.expect(',') && r.integer(&v[1]) && r.expect(',') && r.integer(&v[2]) &&
           r.expect(',') && r.integer(&v[3]) && r.expect(']') && r.expect('}');
      if (!ok) break;
      for (const auto& e : *out) {
        if (e.first == key) {
          r.err = "duplicate key \"" + key + "\"";
          ok = false;
        }
      }
      if (!ok) break;
      out->push_back({key, Tiling{(int)v[0], (int)v[1], (int)v[2], (int)v[3]}});
    } while (r.lit(','));
    ok = ok && r.expect(']');
  }
  ok = ok && r.expect('}');
  if (ok) {
    r.ws();
    if (r.i != text.size()) {
      r.err = "trailing bytes after the document";
      ok = false;
    }
  }
  if (!ok) {
    out->clear();
    *why = r.err.empty() ? "malformed" : r.err;
    return FileState::kCorrupt;
  }
  return FileState::kOk;
}

bool save(const char* path, const Entries& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  bool ok = fprintf(f, "{\"format\": \"glv-autotune-1\", \"entries\": [") > 0;
  for (size_t k = 0; ok && k < entries.size(); ++k) {
    const Tiling& t = entries[k].second;
    ok = fprintf(f, "%s\n  {\"key\": \"%s\", \"tiling\": [%d, %d, %d, %d]}", k ? "," : "", entries[k].first.c_str(),
                 t.block, t.events_per_tile, t.lds_particles, t.pairs_per_round) > 0;
  }
  ok = ok && fprintf(f, "\n]}\n") > 0;
  ok = (fclose(f) == 0) && ok;
  if (ok) ok = rename(tmp.c_str(), path) == 0;
  if (!ok) remove(tmp.c_str());
  return ok;
}

bool lookup_process(const std::string& key, Tiling* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_by_key.find(key);
  if (it == g_by_key.end()) return false;
  *t = it->second;
  return true;
}

void remember_process(const std::string& key, const Tiling& t) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_by_key[key] = t;
}

void forget_process() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_by_key.clear();
}

}  // namespace tune
}  // namespace glv
