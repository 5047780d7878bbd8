// tune_cache.hpp -- the JSON reader of the tuning cache (host only, no HIP),
// kept apart so that it can be checked on the CPU under the address and
// undefined-behaviour sanitizers.
#pragma once

#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

namespace lbdd {
namespace json {

// A small JSON reader for the cache's own format: objects, arrays, strings
// without escapes other than \" and \\, numbers, true, false, null.
struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal *get(const char *key) const {
    for (const auto &kv : obj)
      if (kv.first == key) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char *p, *end;
  int depth = 0;
  void ws() { while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p; }
  bool lit(const char *w) {
    const size_t m = strlen(w);
    if ((size_t)(end - p) < m || strncmp(p, w, m) != 0) return false;
    p += m;
    return true;
  }
  bool string(std::string *out) {
    if (p >= end || *p != '"') return false;
    ++p;
    out->clear();
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (p + 1 >= end || (p[1] != '"' && p[1] != '\\')) return false;
        ++p;
      }
      out->push_back(*p++);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal *v) {
    if (++depth > 16) return false;
    ws();
    if (p >= end) return false;
    bool ok = true;
    if (*p == '{') {
      v->kind = JVal::OBJ;
      ++p;
      ws();
      if (p < end && *p == '}') { ++p; --depth; return true; }
      for (;;) {
        std::string key;
        JVal x;
        ws();
        if (!string(&key)) return false;
        ws();
        if (p >= end || *p++ != ':') return false;
        if (!value(&x)) return false;
        v->obj.emplace_back(key, std::move(x));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == '}') { ++p; break; }
        return false;
      }
    } else if (*p == '[') {
      v->kind = JVal::ARR;
      ++p;
      ws();
      if (p < end && *p == ']') { ++p; --depth; return true; }
      for (;;) {
        JVal x;
        if (!value(&x)) return false;
        v->arr.push_back(std::move(x));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == ']') { ++p; break; }
        return false;
      }
    } else if (*p == '"') {
      v->kind = JVal::STR;
      ok = string(&v->str);
    } else if (lit("true")) {
      v->kind = JVal::BOOL; v->num = 1;
    } else if (lit("false")) {
      v->kind = JVal::BOOL; v->num = 0;
    } else if (lit("null")) {
      v->kind = JVal::NUL;
    } else {
      char buf[64];
      size_t m = 0;
      while (p < end && m < sizeof buf - 1 && (isdigit((unsigned char)*p) || (*p && strchr("+-.eE", *p))))
        buf[m++] = *p++;
      buf[m] = 0;
      char *e = nullptr;
      v->kind = JVal::NUM;
      v->num = strtod(buf, &e);
      ok = m > 0 && e == buf + m && std::isfinite(v->num);
    }
    --depth;
    return ok;
  }
};

// an integer-valued number in [lo, hi]
inline bool jint(const JVal *v, int64_t lo, int64_t hi, int64_t *out) {
  if (!v || v->kind != JVal::NUM || v->num != std::floor(v->num) || v->num < (double)lo || v->num > (double)hi)
    return false;
  *out = (int64_t)v->num;
  return true;
}


}  // namespace json
}  // namespace lbdd
