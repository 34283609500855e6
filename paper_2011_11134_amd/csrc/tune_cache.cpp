// tune_cache.cpp -- the process-wide store of autotuned launch shapes and its
// JSON file.  File format (UTF-8 JSON; unknown fields are ignored):
//   {"format": "dgal-tune-cache", "version": 1,
//    "entries": [{"key": "<arch>/<kind>/K4/fixed1/z1/seg1/b13.6",
//                 "grid": 0, "cull_mult": 16, "exact_mult": 8, "bwd_mult": 0,
//                 "tile_rows": 8, "ms": 0.25}, ...]}
// A file that does not parse, or holds an entry outside the launchable
// ranges, is refused whole.
#include "tune_cache.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/dgal.h"

namespace dgal {

namespace {

struct Entry {
  LaunchShape shape;
  double ms = 0.0;
};

std::mutex store_mu;
std::map<std::string, Entry>& store() {
  static std::map<std::string, Entry>* m = new std::map<std::string, Entry>();
  return *m;
}

// ---- a small JSON reader: values as a tree, enough for the cache format
struct JVal {
  enum Type { kNull, kBool, kNum, kStr, kArr, kObj } type = kNull;
  double num = 0.0;
  bool b = false;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;

  const JVal* get(const char* k) const {
    if (type != kObj) return nullptr;
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct Reader {
  const char* p;
  const char* end;
  int depth = 0;

  void ws() {
    while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
  }
  bool lit(const char* s) {
    const size_t n = strlen(s);
    if ((size_t)(end - p) < n || memcmp(p, s, n) != 0) return false;
    p += n;
    return true;
  }
  bool hex4(unsigned* v) {
    if (end - p < 4) return false;
    *v = 0;
    for (int i = 0; i < 4; ++i) {
      const char c = *p++;
      unsigned d;
      if (c >= '0' && c <= '9') d = (unsigned)(c - '0');
      else if (c >= 'a' && c <= 'f') d = (unsigned)(c - 'a' + 10);
      else if (c >= 'A' && c <= 'F') d = (unsigned)(c - 'A' + 10);
      else return false;
      *v = *v * 16 + d;
    }
    return true;
  }
  bool string(std::string* out) {
    if (p >= end || *p != '"') return false;
    ++p;
    out->clear();
    while (p < end && *p != '"') {
      char c = *p++;
      if ((unsigned char)c < 0x20) return false;
      if (c == '\\') {
        if (p >= end) return false;
        c = *p++;
        switch (c) {
          case '"': case '\\': case '/': out->push_back(c); break;
          case 'b': out->push_back('\b'); break;
          case 'f': out->push_back('\f'); break;
          case 'n': out->push_back('\n'); break;
          case 'r': out->push_back('\r'); break;
          case 't': out->push_back('\t'); break;
          case 'u': {
            unsigned v;
            if (!hex4(&v)) return false;
            if (v >= 0x80) return false;  // keys and names are ASCII
            out->push_back((char)v);
            break;
          }
          default: return false;
        }
      } else {
        out->push_back(c);
      }
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool number(double* out) {
    const char* s = p;
    if (p < end && *p == '-') ++p;
    if (p >= end || !(*p >= '0' && *p <= '9')) return false;
    while (p < end && ((*p >= '0' && *p <= '9') || *p == '.' || *p == 'e' || *p == 'E' ||
                       *p == '+' || *p == '-'))
      ++p;
    const std::string t(s, (size_t)(p - s));
    char* e = nullptr;
    *out = strtod(t.c_str(), &e);
    return e != nullptr && *e == '\0';
  }
  bool value(JVal* v) {
    ws();
    if (p >= end || ++depth > 32) return false;
    bool ok = false;
    if (*p == '{') {
      ++p;
      v->type = JVal::kObj;
      ws();
      if (p < end && *p == '}') {
        ++p;
        ok = true;
      } else {
        while (true) {
          ws();
          std::pair<std::string, JVal> kv;
          if (!string(&kv.first)) break;
          ws();
          if (p >= end || *p != ':') break;
          ++p;
          if (!value(&kv.second)) break;
          v->obj.push_back(std::move(kv));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == '}') { ++p; ok = true; }
          break;
        }
      }
    } else if (*p == '[') {
      ++p;
      v->type = JVal::kArr;
      ws();
      if (p < end && *p == ']') {
        ++p;
        ok = true;
      } else {
        while (true) {
          JVal e;
          if (!value(&e)) break;
          v->arr.push_back(std::move(e));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == ']') { ++p; ok = true; }
          break;
        }
      }
    } else if (*p == '"') {
      v->type = JVal::kStr;
      ok = string(&v->str);
    } else if (lit("true")) {
      v->type = JVal::kBool;
      v->b = true;
      ok = true;
    } else if (lit("false")) {
      v->type = JVal::kBool;
      ok = true;
    } else if (lit("null")) {
      ok = true;
    } else {
      v->type = JVal::kNum;
      ok = number(&v->num);
    }
    --depth;
    return ok;
  }
};

// An integer field in [lo, hi] (absent: 0, which every field accepts).
bool int_field(const JVal& o, const char* k, int64_t lo, int64_t hi, int64_t* out) {
  const JVal* v = o.get(k);
  if (v == nullptr) {
    *out = 0;
    return true;
  }
  if (v->type != JVal::kNum || !(v->num >= (double)lo && v->num <= (double)hi)) return false;
  const int64_t i = (int64_t)v->num;
  if ((double)i != v->num) return false;
  *out = i;
  return true;
}

bool key_valid(const std::string& k) {
  if (k.empty() || k.size() > 200) return false;
  for (char c : k)
    if (!((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9') ||
          c == '_' || c == '/' || c == '.' || c == '-' || c == ':' || c == '+'))
      return false;
  return true;
}

}  // namespace

bool shape_valid(const LaunchShape& s) {
  return s.grid >= 0 && s.grid <= (1 << 24) && s.cull_mult >= 0 && s.cull_mult <= 64 &&
         s.exact_mult >= 0 && s.exact_mult <= 64 && s.bwd_mult >= 0 && s.bwd_mult <= 64 &&
         (s.tile_rows == 0 || s.tile_rows == 4 || s.tile_rows == 8 || s.tile_rows == 16);
}

bool tune_store_get(const std::string& key, LaunchShape* out) {
  std::lock_guard<std::mutex> lock(store_mu);
  const auto it = store().find(key);
  if (it == store().end()) return false;
  *out = it->second.shape;
  return true;
}

void tune_store_put(const std::string& key, const LaunchShape& s, double ms) {
  std::lock_guard<std::mutex> lock(store_mu);
  Entry& e = store()[key];
  e.shape = s;
  e.ms = ms;
}

void tune_store_clear() {
  std::lock_guard<std::mutex> lock(store_mu);
  store().clear();
}

int64_t tune_store_size() {
  std::lock_guard<std::mutex> lock(store_mu);
  return (int64_t)store().size();
}

int tune_store_load(const char* path) {
  if (path == nullptr || path[0] == '\0') return DGAL_EINVAL;
  FILE* f = fopen(path, "rb");
  if (f == nullptr) return DGAL_EIO;
  std::string text;
  char buf[4096];
  size_t n;
  bool too_big = false;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, n);
    if (text.size() > (16u << 20)) {
      too_big = true;
      break;
    }
  }
  const bool read_err = ferror(f) != 0;
  fclose(f);
  if (read_err) return DGAL_EIO;
  if (too_big) return DGAL_EINVAL;
  Reader r{text.data(), text.data() + text.size()};
  JVal root;
  if (!r.value(&root)) return DGAL_EINVAL;
  r.ws();
  if (r.p != r.end || root.type != JVal::kObj) return DGAL_EINVAL;
  const JVal* fmt = root.get("format");
  const JVal* ver = root.get("version");
  const JVal* ents = root.get("entries");
  if (fmt == nullptr || fmt->type != JVal::kStr || fmt->str != "dgal-tune-cache") return DGAL_EINVAL;
  if (ver == nullptr || ver->type != JVal::kNum || ver->num != 1.0) return DGAL_EINVAL;
  if (ents == nullptr || ents->type != JVal::kArr) return DGAL_EINVAL;
  std::vector<std::pair<std::string, Entry>> got;
  for (const JVal& e : ents->arr) {
    if (e.type != JVal::kObj) return DGAL_EINVAL;
    const JVal* key = e.get("key");
    if (key == nullptr || key->type != JVal::kStr || !key_valid(key->str)) return DGAL_EINVAL;
    int64_t grid, cull, exact, bwd, rows;
    if (!int_field(e, "grid", 0, 1 << 24, &grid) || !int_field(e, "cull_mult", 0, 64, &cull) ||
        !int_field(e, "exact_mult", 0, 64, &exact) || !int_field(e, "bwd_mult", 0, 64, &bwd) ||
        !int_field(e, "tile_rows", 0, 16, &rows))
      return DGAL_EINVAL;
    Entry en;
    en.shape.grid = grid;
    en.shape.cull_mult = (int)cull;
    en.shape.exact_mult = (int)exact;
    en.shape.bwd_mult = (int)bwd;
    en.shape.tile_rows = (int)rows;
    if (!shape_valid(en.shape)) return DGAL_EINVAL;
    const JVal* ms = e.get("ms");
    if (ms != nullptr) {
      if (ms->type != JVal::kNum || !(ms->num >= 0.0 && ms->num < 1e9)) return DGAL_EINVAL;
      en.ms = ms->num;
    }
    got.emplace_back(key->str, en);
  }
  std::lock_guard<std::mutex> lock(store_mu);
  for (auto& kv : got) store()[kv.first] = kv.second;
  return (int)got.size();
}

int tune_store_save(const char* path) {
  if (path == nullptr || path[0] == '\0') return DGAL_EINVAL;
  std::string out = "{\"format\": \"dgal-tune-cache\", \"version\": 1, \"entries\": [";
  {
    std::lock_guard<std::mutex> lock(store_mu);
    bool first = true;
    for (const auto& kv : store()) {
      const LaunchShape& s = kv.second.shape;
      char line[512];
      snprintf(line, sizeof(line),
               "%s\n {\"key\": \"%s\", \"grid\": %lld, \"cull_mult\": %d, \"exact_mult\": %d, "
               "\"bwd_mult\": %d, \"tile_rows\": %d, \"ms\": %.6f}",
               first ? "" : ",", kv.first.c_str(), (long long)s.grid, s.cull_mult, s.exact_mult,
               s.bwd_mult, s.tile_rows, kv.second.ms);
      out += line;
      first = false;
    }
  }
  out += "\n]}\n";
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
  FILE* f = fopen(tmp.c_str(), "wb");
  if (f == nullptr) return DGAL_EIO;
  const bool ok = fwrite(out.data(), 1, out.size(), f) == out.size();
  const bool closed = fclose(f) == 0;
  if (!ok || !closed || rename(tmp.c_str(), path) != 0) {
    remove(tmp.c_str());
    return DGAL_EIO;
  }
  return DGAL_OK;
}

int tune_store_report(char* buf, int64_t size) {
  std::lock_guard<std::mutex> lock(store_mu);
  int64_t used = 0;
  if (size > 0) buf[0] = '\0';
  for (const auto& kv : store()) {
    const LaunchShape& s = kv.second.shape;
    char line[400];
    const int n = snprintf(line, sizeof(line), "%s grid=%lld cull=%d exact=%d bwd=%d rows=%d ms=%.6f\n",
                           kv.first.c_str(), (long long)s.grid, s.cull_mult, s.exact_mult,
                           s.bwd_mult, s.tile_rows, kv.second.ms);
    if (n > 0 && used + n < size) {
      memcpy(buf + used, line, (size_t)n + 1);
      used += n;
    }
  }
  return (int)store().size();
}

const char* tune_cache_path() {
  static std::once_flag once;
  static std::string path;
  std::call_once(once, [] {
    const char* p = getenv("DGAL_TUNE_CACHE");
    if (p == nullptr || p[0] == '\0') return;
    // a missing file is created by the first save; a file that exists but
    // does not load as a cache is never overwritten (the cache is then off)
    if (access(p, F_OK) == 0 && tune_store_load(p) < 0) return;
    path = p;
  });
  return path.empty() ? nullptr : path.c_str();
}

}  // namespace dgal
