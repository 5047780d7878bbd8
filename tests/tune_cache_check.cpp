// CPU checks of the tuning cache's JSON reader (no GPU, no HIP), built with
// the address and undefined-behaviour sanitizers: well-formed documents parse
// to the values written, malformed ones are refused, and random damage to a
// document never reads out of bounds.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "../paper_2304_06543_amd/csrc/tune_cache.hpp"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++failures; } \
  } while (0)

using lbdd::json::JParser;
using lbdd::json::JVal;

static bool parse(const std::string &t, JVal *v) {
  JParser p{t.data(), t.data() + t.size()};
  if (!p.value(v)) return false;
  p.ws();
  return p.p == p.end;
}

int main() {
  const std::string doc =
      "{\"format\": \"lbdd-tune-1\", \"entries\": [\n"
      "  {\"arch\": \"gfx950\", \"kind\": \"search\", \"k_bucket\": 7, \"n_bucket\": 5, \"ratio\": -1},\n"
      "  {\"arch\": \"gfx950\", \"kind\": \"scan\", \"k\": 500, \"vec4\": 1, \"config\": [4, 64, 2, 1]}\n]}\n";
  {
    JVal v;
    CHECK(parse(doc, &v));
    CHECK(v.kind == JVal::OBJ);
    const JVal *e = v.get("entries");
    CHECK(e && e->kind == JVal::ARR && e->arr.size() == 2);
    int64_t x = 0;
    CHECK(lbdd::json::jint(e->arr[0].get("ratio"), -1, 1 << 20, &x) && x == -1);
    CHECK(!lbdd::json::jint(e->arr[0].get("ratio"), 0, 1 << 20, &x));
    const JVal *c = e->arr[1].get("config");
    CHECK(c && c->kind == JVal::ARR && c->arr.size() == 4);
    CHECK(lbdd::json::jint(&c->arr[1], 1, 64, &x) && x == 64);
    CHECK(e->arr[1].get("arch")->str == "gfx950");
    CHECK(!e->arr[1].get("missing"));
  }
  {  // literals, escapes, empty containers, nesting
    JVal v;
    CHECK(parse("[true, false, null, \"a\\\"b\\\\c\", [], {}, -2.5e3]", &v));
    CHECK(v.arr.size() == 7 && v.arr[3].str == "a\"b\\c" && v.arr[6].num == -2500.0);
  }
  const char *bad[] = {"", "{", "[1,]", "{\"a\" 1}", "{\"a\": }", "\"open", "\"bad\\n escape\"", "nul",
                       "[1 2]", "{1: 2}", "1e999", "--1", "[[[[[[[[[[[[[[[[[[[[1]]]]]]]]]]]]]]]]]]]"};
  for (const char *b : bad) {
    JVal v;
    CHECK(!parse(b, &v));
  }
  {  // numbers must be whole and in range to count as integers
    JVal v;
    int64_t x;
    CHECK(parse("[1.5, 1e2, 7]", &v));
    CHECK(!lbdd::json::jint(&v.arr[0], 0, 10, &x));
    CHECK(lbdd::json::jint(&v.arr[1], 0, 100, &x) && x == 100);
    CHECK(!lbdd::json::jint(&v.arr[2], 8, 10, &x));
    CHECK(!lbdd::json::jint(nullptr, 0, 10, &x));
  }
  {  // random damage: truncation, byte flips, embedded NULs
    srand(11);
    for (int t = 0; t < 20000; ++t) {
      std::string d = doc;
      const int edits = 1 + rand() % 4;
      for (int e = 0; e < edits; ++e) {
        const size_t at = (size_t)rand() % d.size();
        switch (rand() % 3) {
          case 0: d.resize(at); break;
          case 1: d[at] = (char)(rand() % 256); break;
          default: d.insert(at, 1, (char)(rand() % 256));
        }
        if (d.empty()) d = "x";
      }
      JVal v;
      (void)parse(d, &v);            // accepted or refused, never out of bounds
    }
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
