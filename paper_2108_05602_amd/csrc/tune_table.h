// Process-wide table of tuned launch configurations of the fused search
// (internal to libfringe), and its JSON file form.
#pragma once

#include <string>

namespace fringe {

// A class of bands the tuner times on its own: the device kind and the
// search shape that select the kernels.
struct TuneKey {
  std::string arch;      // device architecture name (e.g. gfx950)
  int cus = 0;           // compute units
  int n_freq = 0;        // F = n_if * n_chan
  int pad_freq = 0;
  int pad_time = 0;      // 0: the delay-only search
  int log2_wmax = 0;     // longest window (<= 64 APs)
};

// The tuned choice and the timings behind it.
struct TuneVal {
  int spectra = 0;       // 1: delay spectra through HBM, then the rate kernels
  int chunk = 0;         // APs per work item
  float ms_fused = -1.f;    // best sample time of each mode (< 0: not a candidate)
  float ms_spectra = -1.f;
};

bool tune_lookup(const TuneKey& k, TuneVal* v);
void tune_store(const TuneKey& k, const TuneVal& v);
void tune_clear();
// 0 on success, else -1 with *err set.
int tune_save(const char* path, std::string* err);
// Entries of the file are merged into the table (replacing equal keys).
int tune_load(const char* path, std::string* err);

}  // namespace fringe
