// Tuned launch parameters read by the library itself, so that a C caller
// gets the autotuner's shapes without any Python: the JSON cache written by
// paper_2207_00257_amd/tune.py (tuned/plain.json next to libnrm.so, or the
// file named by $NRM_TUNE_CACHE), keyed "arch/in->out/accum/2^k" with k =
// floor(log2 n). A context whose parameters were never set explicitly takes
// the entry of each call's key when there is one, its own defaults otherwise.
//
// The reader handles the cache's shape only: an object of entries, each an
// object whose "params" member maps field names to integers; other members
// and values are skipped.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "nrm_ctx.h"

namespace {

using Fields = std::map<std::string, int64_t>;

class Reader {
 public:
  explicit Reader(const std::string& s) : s_(s) {}
  bool parse(std::map<std::string, Fields>* out) {
    ws();
    if (!eat('{')) return false;
    ws();
    if (eat('}')) return true;
    while (true) {
      std::string key;
      if (!str(&key)) return false;
      ws();
      if (!eat(':')) return false;
      ws();
      Fields f;
      if (!entry(&f)) return false;
      (*out)[key] = f;
      ws();
      if (eat(',')) {
        ws();
        continue;
      }
      return eat('}');
    }
  }

 private:
  const std::string& s_;
  size_t i_ = 0;

  void ws() {
    while (i_ < s_.size() && std::isspace((unsigned char)s_[i_])) ++i_;
  }
  bool eat(char c) {
    if (i_ < s_.size() && s_[i_] == c) {
      ++i_;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    if (!eat('"')) return false;
    while (i_ < s_.size() && s_[i_] != '"') {
      if (s_[i_] == '\\' && i_ + 1 < s_.size()) ++i_;
      out->push_back(s_[i_++]);
    }
    return eat('"');
  }
  bool number(double* v) {
    const char* b = s_.c_str() + i_;
    char* e = nullptr;
    *v = std::strtod(b, &e);
    if (e == b) return false;
    i_ += (size_t)(e - b);
    return true;
  }
  // Skips any value.
  bool skip() {
    ws();
    if (i_ >= s_.size()) return false;
    const char c = s_[i_];
    if (c == '"') {
      std::string t;
      return str(&t);
    }
    if (c == '{' || c == '[') {
      const char close = c == '{' ? '}' : ']';
      ++i_;
      ws();
      if (eat(close)) return true;
      while (true) {
        if (c == '{') {
          std::string k;
          if (!str(&k)) return false;
          ws();
          if (!eat(':')) return false;
        }
        if (!skip()) return false;
        ws();
        if (eat(',')) {
          ws();
          continue;
        }
        return eat(close);
      }
    }
    if (s_.compare(i_, 4, "true") == 0 || s_.compare(i_, 4, "null") == 0) {
      i_ += 4;
      return true;
    }
    if (s_.compare(i_, 5, "false") == 0) {
      i_ += 5;
      return true;
    }
    double v;
    return number(&v);
  }
  // One entry: its "params" object's integer members.
  bool entry(Fields* f) {
    if (!eat('{')) return skip();
    ws();
    if (eat('}')) return true;
    while (true) {
      std::string k;
      if (!str(&k)) return false;
      ws();
      if (!eat(':')) return false;
      ws();
      if (k == "params" && eat('{')) {
        ws();
        if (!eat('}')) {
          while (true) {
            std::string name;
            if (!str(&name)) return false;
            ws();
            if (!eat(':')) return false;
            ws();
            double v;
            if (number(&v)) (*f)[name] = (int64_t)v;
            else if (!skip()) return false;
            ws();
            if (eat(',')) {
              ws();
              continue;
            }
            if (!eat('}')) return false;
            break;
          }
        }
      } else if (!skip()) {
        return false;
      }
      ws();
      if (eat(',')) {
        ws();
        continue;
      }
      return eat('}');
    }
  }
};

std::once_flag g_once;
std::map<std::string, Fields>* g_cache = nullptr;

std::string default_path() {
  if (const char* env = std::getenv("NRM_TUNE_CACHE")) return env;
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&nrm_normalize_ex), &info) && info.dli_fname) {
    std::string lib = info.dli_fname;
    const size_t slash = lib.rfind('/');
    return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuned/plain.json";
  }
  return "";
}

const std::map<std::string, Fields>& cache() {
  std::call_once(g_once, [] {
    g_cache = new std::map<std::string, Fields>();
    const std::string path = default_path();
    if (path.empty()) return;
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    std::map<std::string, Fields> parsed;
    if (Reader(text).parse(&parsed)) g_cache->swap(parsed);  // a malformed file counts as empty
  });
  return *g_cache;
}

const char* dt_name(int dt) { return dt == NRM_F32 ? "f32" : dt == NRM_BF16 ? "bf16" : "f16"; }

bool set_field(nrm_params* p, const std::string& k, int64_t v) {
  struct F {
    const char* name;
    int32_t nrm_params::*m;
  };
  static const F fields[] = {
      {"block", &nrm_params::block},           {"unroll", &nrm_params::unroll},
      {"grid", &nrm_params::grid},             {"layout", &nrm_params::layout},
      {"reduce_nt", &nrm_params::reduce_nt},   {"max_height", &nrm_params::max_height},
      {"map_block", &nrm_params::map_block},   {"map_unroll", &nrm_params::map_unroll},
      {"map_grid", &nrm_params::map_grid},     {"map_layout", &nrm_params::map_layout},
      {"map_nt", &nrm_params::map_nt},         {"reverse_map", &nrm_params::reverse_map},
      {"reduce_keep_mib", &nrm_params::reduce_keep_mib}, {"tile_log2", &nrm_params::tile_log2},
      {"fused_combine", &nrm_params::fused_combine},     {"small_n", &nrm_params::small_n},
      {"resident_n", &nrm_params::resident_n},
  };
  for (const F& f : fields)
    if (k == f.name) {
      p->*f.m = (int32_t)v;
      return true;
    }
  return false;
}

}  // namespace

namespace nrm {

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

bool tuned_plain(const std::string& arch, int in_dt, int out_dt, int acc, int64_t n, nrm_params* p) {
  int k = 0;
  while ((int64_t(1) << (k + 1)) <= n && k < 62) ++k;
  const std::string key = arch + "/" + dt_name(in_dt) + "->" + dt_name(out_dt) + "/" +
                          (acc == NRM_ACC_KAHAN ? "kahan" : "f32") + "/2^" + std::to_string(k);
  const auto& c = cache();
  auto it = c.find(key);
  if (it == c.end()) return false;
  nrm_params q = *p;
  for (const auto& kv : it->second)
    if (!set_field(&q, kv.first, kv.second)) return false;  // a field this library does not know
  *p = q;
  return true;
}

}  // namespace nrm

extern "C" int nrm_tuned_params(const char* arch, int in_dtype, int out_dtype, int accum, int64_t n,
                                nrm_params* params) {
  if (!arch || !params) return nrm::fail(NRM_EINVAL, "NULL argument");
  if (n < 1) return nrm::fail(NRM_EINVAL, "n must be positive");
  auto ok_dt = [](int dt) { return dt == NRM_F32 || dt == NRM_BF16 || dt == NRM_F16; };
  if (!ok_dt(in_dtype) || !ok_dt(out_dtype)) return nrm::fail(NRM_EINVAL, "unknown dtype");
  if (accum != NRM_ACC_F32 && accum != NRM_ACC_KAHAN) return nrm::fail(NRM_EINVAL, "unknown accumulation mode");
  nrm_default_params(params);
  return nrm::tuned_plain(arch, in_dtype, out_dtype, accum, n, params) ? 1 : 0;
}
