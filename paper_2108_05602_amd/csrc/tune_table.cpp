// The tune table and its JSON file (see tune_table.h).  The file is an
// object {"fringe_tune_table": 1, "entries": [ {...}, ... ]} with one flat
// object per entry; the reader accepts any whitespace and key order and
// ignores unknown keys.
#include "tune_table.h"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <vector>

namespace fringe {

namespace {

std::mutex g_mu;
std::vector<std::pair<TuneKey, TuneVal>> g_table;

bool same(const TuneKey& a, const TuneKey& b) {
  return a.arch == b.arch && a.cus == b.cus && a.n_freq == b.n_freq && a.pad_freq == b.pad_freq &&
         a.pad_time == b.pad_time && a.log2_wmax == b.log2_wmax;
}

void store_locked(const TuneKey& k, const TuneVal& v) {
  for (auto& e : g_table)
    if (same(e.first, k)) {
      e.second = v;
      return;
    }
  g_table.emplace_back(k, v);
}

// Minimal reader for the flat objects of the file.
struct Reader {
  const std::string& s;
  size_t i = 0;
  explicit Reader(const std::string& text) : s(text) {}
  void ws() {
    while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool num(double* out) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    *out = std::strtod(b, &e);
    if (e == b) return false;
    i += size_t(e - b);
    return true;
  }
};

}  // namespace

bool tune_lookup(const TuneKey& k, TuneVal* v) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (const auto& e : g_table)
    if (same(e.first, k)) {
      *v = e.second;
      return true;
    }
  return false;
}

void tune_store(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> lock(g_mu);
  store_locked(k, v);
}

void tune_clear() {
  std::lock_guard<std::mutex> lock(g_mu);
  g_table.clear();
}

int tune_save(const char* path, std::string* err) {
  std::vector<std::pair<TuneKey, TuneVal>> copy;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    copy = g_table;
  }
  std::ostringstream o;
  o << "{\"fringe_tune_table\": 1, \"entries\": [";
  for (size_t n = 0; n < copy.size(); ++n) {
    const TuneKey& k = copy[n].first;
    const TuneVal& v = copy[n].second;
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "%s\n  {\"arch\": \"%s\", \"cus\": %d, \"n_freq\": %d, \"pad_freq\": %d, "
                  "\"pad_time\": %d, \"log2_wmax\": %d, \"spectra\": %d, \"chunk\": %d, "
                  "\"ms_fused\": %.9g, \"ms_spectra\": %.9g}",
                  n ? "," : "", k.arch.c_str(), k.cus, k.n_freq, k.pad_freq, k.pad_time,
                  k.log2_wmax, v.spectra, v.chunk, double(v.ms_fused), double(v.ms_spectra));
    o << buf;
  }
  o << "\n]}\n";
  std::ofstream f(path, std::ios::binary | std::ios::trunc);
  if (!f) {
    *err = std::string("cannot open ") + path + " for writing";
    return -1;
  }
  f << o.str();
  if (!f) {
    *err = std::string("write to ") + path + " failed";
    return -1;
  }
  return 0;
}

int tune_load(const char* path, std::string* err) {
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    *err = std::string("cannot open ") + path;
    return -1;
  }
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  const size_t at = text.find("\"entries\"");
  if (text.find("\"fringe_tune_table\"") == std::string::npos || at == std::string::npos) {
    *err = std::string(path) + " is not a tune table";
    return -1;
  }
  Reader r(text);
  r.i = at + 9;
  if (!r.eat(':') || !r.eat('[')) {
    *err = std::string(path) + ": \"entries\" is not a list";
    return -1;
  }
  std::vector<std::pair<TuneKey, TuneVal>> got;
  if (!r.eat(']')) {
    do {
      if (!r.eat('{')) {
        *err = std::string(path) + ": an entry is not an object";
        return -1;
      }
      TuneKey k;
      TuneVal v;
      int seen = 0;
      if (!r.eat('}')) {
        do {
          std::string key;
          if (!r.str(&key) || !r.eat(':')) {
            *err = std::string(path) + ": malformed entry";
            return -1;
          }
          if (key == "arch") {
            if (!r.str(&k.arch)) {
              *err = std::string(path) + ": arch is not a string";
              return -1;
            }
            ++seen;
            continue;
          }
          double x = 0;
          if (!r.num(&x)) {
            *err = std::string(path) + ": value of " + key + " is not a number";
            return -1;
          }
          const int xi = static_cast<int>(x);
          if (key == "cus") k.cus = xi, ++seen;
          else if (key == "n_freq") k.n_freq = xi, ++seen;
          else if (key == "pad_freq") k.pad_freq = xi, ++seen;
          else if (key == "pad_time") k.pad_time = xi, ++seen;
          else if (key == "log2_wmax") k.log2_wmax = xi, ++seen;
          else if (key == "spectra") v.spectra = xi ? 1 : 0, ++seen;
          else if (key == "chunk") v.chunk = xi, ++seen;
          else if (key == "ms_fused") v.ms_fused = float(x);
          else if (key == "ms_spectra") v.ms_spectra = float(x);
        } while (r.eat(','));
        if (!r.eat('}')) {
          *err = std::string(path) + ": unterminated entry";
          return -1;
        }
      }
      if (seen < 8 || v.chunk < 1) {
        *err = std::string(path) + ": an entry lacks a field";
        return -1;
      }
      got.emplace_back(k, v);
    } while (r.eat(','));
    if (!r.eat(']')) {
      *err = std::string(path) + ": unterminated entry list";
      return -1;
    }
  }
  std::lock_guard<std::mutex> lock(g_mu);
  for (const auto& e : got) store_locked(e.first, e.second);
  return 0;
}

}  // namespace fringe
