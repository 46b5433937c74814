// Launch-shape tuning per class of graph (the degree-binning thresholds and
// grid caps that replace the paper's OpenMP dynamic schedule, Sec. 4.1).
//
// The table holds one gvl_tuning per class.  It starts from the compiled
// defaults, is loaded once per process from a tune file (written by
// paper_2312_13936_amd/tune.py) when the first context is created, and can
// be changed at run time with gvl_set_tuning.  Every value only changes
// which kernel handles a row or how many workgroups a launch uses, never a
// result: the bin limits stay within the compiled ones.
//
// Tune file: one line per class, "<class> b0 b1 b2 b3 b4 b5 decide_grid
// commit_grid agg_grid" with class one of small, lowdeg, skewed, batch;
// '#' starts a comment.  Its path is $GVL_TUNE_FILE if set (the value
// "none" skips loading), else tune.txt next to libgvl.so.
#include <dlfcn.h>

#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

#include "host.hpp"

namespace {

const char* const kClassNames[GVL_NUM_CLASSES] = {"small", "lowdeg", "skewed", "batch"};

gvl_tuning compiled_default() {
  gvl_tuning t;
  for (int b = 0; b < kTunedBins; ++b) t.bin_max[b] = kBinMax[b];
  t.decide_grid = 1024;  // measured best on R-MAT scale 24 (four workgroups per CU)
  t.commit_grid = 2048;
  t.agg_grid = 4096;
  return t;
}

std::mutex g_mu;
gvl_tuning g_table[GVL_NUM_CLASSES] = {compiled_default(), compiled_default(), compiled_default(),
                                       compiled_default()};
std::once_flag g_loaded;

bool valid(const gvl_tuning& t) {
  int32_t prev = 1;
  for (int b = 0; b < kTunedBins; ++b) {
    if (t.bin_max[b] < prev || t.bin_max[b] > kBinMax[b]) return false;
    prev = t.bin_max[b];
  }
  if (t.bin_max[kTunedBins - 1] < kMinBin5) return false;
  for (int32_t g : {t.decide_grid, t.commit_grid, t.agg_grid})
    if (g < 1 || g > 65536) return false;
  return true;
}

std::string default_path() {
  const char* env = std::getenv("GVL_TUNE_FILE");
  if (env) return std::string(env);
  Dl_info info;
  if (dladdr((void*)&compiled_default, &info) && info.dli_fname) {
    std::string so(info.dli_fname);
    const size_t slash = so.rfind('/');
    return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune.txt";
  }
  return "tune.txt";
}

gvl_status load_file(const std::string& path, bool quiet_if_missing) {
  std::ifstream f(path);
  if (!f) return quiet_if_missing ? GVL_OK : GVL_E_INVALID_ARG;
  gvl_tuning next[GVL_NUM_CLASSES];
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (int c = 0; c < GVL_NUM_CLASSES; ++c) next[c] = g_table[c];
  }
  std::string line;
  int lineno = 0;
  while (std::getline(f, line)) {
    ++lineno;
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream in(line);
    std::string name;
    if (!(in >> name)) continue;
    int cls = -1;
    for (int c = 0; c < GVL_NUM_CLASSES; ++c)
      if (name == kClassNames[c]) cls = c;
    gvl_tuning t;
    bool ok = cls >= 0;
    for (int b = 0; ok && b < kTunedBins; ++b) ok = static_cast<bool>(in >> t.bin_max[b]);
    ok = ok && (in >> t.decide_grid >> t.commit_grid >> t.agg_grid) && valid(t);
    if (!ok) {
      fprintf(stderr, "gvl: %s:%d: tuning line ignored\n", path.c_str(), lineno);
      continue;
    }
    next[cls] = t;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  for (int c = 0; c < GVL_NUM_CLASSES; ++c) g_table[c] = next[c];
  return GVL_OK;
}

}  // namespace

// Loads the tune file once per process (from gvl_create).
void gvl_tuning_load_once() {
  std::call_once(g_loaded, [] {
    const std::string p = default_path();
    if (p != "none") (void)load_file(p, true);
  });
}

int32_t gvl_class_of(int64_t n, int64_t m, bool fused) {
  if (fused) return GVL_CLASS_BATCH;
  if (n <= 131072) return GVL_CLASS_SMALL;
  if (m < 6 * n) return GVL_CLASS_LOWDEG;
  return GVL_CLASS_SKEWED;
}

gvl_tuning gvl_tuning_of(int32_t cls) {
  std::lock_guard<std::mutex> lock(g_mu);
  return g_table[(cls >= 0 && cls < GVL_NUM_CLASSES) ? cls : GVL_CLASS_SKEWED];
}

BinLimits bin_limits(const gvl_tuning& t) {
  BinLimits lim;
  for (int b = 0; b < kNumBins; ++b) lim.v[b] = (b < kTunedBins) ? t.bin_max[b] : kBinMax[b];
  return lim;
}

extern "C" {

gvl_status gvl_graph_class(int64_t n, int64_t m, int32_t fused, int32_t* cls) {
  if (!cls || n < 0 || m < 0) return GVL_E_INVALID_ARG;
  *cls = gvl_class_of(n, m, fused != 0);
  return GVL_OK;
}

gvl_status gvl_get_tuning(int32_t cls, gvl_tuning* t) {
  if (!t || cls < 0 || cls >= GVL_NUM_CLASSES) return GVL_E_INVALID_ARG;
  gvl_tuning_load_once();
  *t = gvl_tuning_of(cls);
  return GVL_OK;
}

gvl_status gvl_set_tuning(int32_t cls, const gvl_tuning* t) {
  if (!t || cls < 0 || cls >= GVL_NUM_CLASSES || !valid(*t)) return GVL_E_INVALID_ARG;
  gvl_tuning_load_once();
  std::lock_guard<std::mutex> lock(g_mu);
  g_table[cls] = *t;
  return GVL_OK;
}

gvl_status gvl_load_tuning(const char* path) {
  if (!path) return GVL_E_INVALID_ARG;
  gvl_tuning_load_once();
  return load_file(path, false);
}

}  // extern "C"
