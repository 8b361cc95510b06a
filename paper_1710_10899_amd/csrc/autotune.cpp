// Tuning table for the persistent large-order launches.
//
// The table maps an upper bound on the submatrix order to a launch
// parameter, by kind:
//   0 / 1  workgroups per compute unit of the FP32 / FP64 persistent kernels
//   2      workgroups per compute unit of the tridiagonal eigensolver
//          (capped by its LDS use at launch)
//   3 / 4  panel width of the FP64 / FP32 tridiagonal reduction (even, 2..48)
//   5 / 6  workgroups per compute unit the FP64 / FP32 reduction is laid
//          out for (1..4: its LDS panel copy takes the rest of the share)
//   7      largest order of the one-wavefront bucket (1..64; m_hi unused),
//          the edge between the one-sided Jacobi and the reduction path (32:
//          on overlap workloads of orders 13..117 the reduction path is the
//          faster one from order 39 on, forward + adjoint 14.9 against 33.8 ms
//          with the edge at 64)
// Defaults are the gfx950 measurements on the overlap workloads (the FP32
// reduction runs three workgroups per compute unit: 118.5 against 137.0 ms
// with two on the 6656-column workload, 869 against 981 ms on 26,624 columns
// of order ~500; the FP64 one two: three spill and were slower); a file
// written by the package's autotune script (environment variable
// SUBMAT_TUNE_FILE, lines "kind m_hi value") overrides them.
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "autotune.hpp"

namespace submat {
namespace {

struct Entry {
  int fp64, m_hi, bpc;
};

std::vector<Entry> g_table;
bool g_loaded = false;
bool g_from_file = false;
std::mutex g_tmu;

void load_locked(bool use_file) {
  g_table = {{1, 128, 8}, {1, 256, 4}, {1, 1024, 2}, {1, 1 << 30, 1},
             {0, 128, 8}, {0, 256, 4}, {0, 1024, 2}, {0, 1 << 30, 1},
             {2, 256, 8}, {2, 512, 6}, {2, 1024, 4}, {2, 1 << 30, 1},
             {3, 1 << 30, 16}, {4, 1 << 30, 16}, {5, 1 << 30, 2}, {6, 1 << 30, 3},
             {7, 1 << 30, 32}};
  g_from_file = false;
  const char* path = use_file ? std::getenv("SUBMAT_TUNE_FILE") : nullptr;
  if (path && *path) {
    if (FILE* f = std::fopen(path, "r")) {
      std::vector<Entry> t;
      Entry e;
      while (std::fscanf(f, "%d %d %d", &e.fp64, &e.m_hi, &e.bpc) == 3) {
        bool ok = e.m_hi >= 1 && e.fp64 >= 0 && e.fp64 <= 7;
        if (e.fp64 <= 2) ok = ok && e.bpc >= 1 && e.bpc <= 32;
        else if (e.fp64 <= 4) ok = ok && e.bpc >= 2 && e.bpc <= 48 && !(e.bpc & 1);
        else if (e.fp64 <= 6) ok = ok && e.bpc >= 1 && e.bpc <= 4;
        else ok = ok && e.bpc >= 1 && e.bpc <= 64;
        if (ok) t.push_back(e);
      }
      std::fclose(f);
      if (!t.empty()) {
        g_table = t;
        g_from_file = true;
      }
    }
  }
  g_loaded = true;
}

}  // namespace

void reload_tuning(bool use_file) {
  std::lock_guard<std::mutex> lk(g_tmu);
  load_locked(use_file);
}

bool tuning_from_file() {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_loaded) load_locked(true);
  return g_from_file;
}

static int lookup(int kind, int max_m, int fallback = 1) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_loaded) load_locked(true);
  int best = fallback, best_hi = 1 << 30;
  bool found = false;
  for (const Entry& e : g_table) {
    if (e.fp64 != kind || max_m > e.m_hi) continue;
    if (!found || e.m_hi < best_hi) {
      best = e.bpc;
      best_hi = e.m_hi;
      found = true;
    }
  }
  return best;
}

int tuned_blocks_per_cu(int max_m, int fp64) { return lookup(fp64 ? 1 : 0, max_m); }

int tuned_eig_blocks_per_cu(int max_m) { return lookup(2, max_m); }

int tuned_reduction_nb(int max_m, int fp64) { return lookup(fp64 ? 3 : 4, max_m, 16); }

int tuned_reduction_per_cu(int max_m, int fp64) { return lookup(fp64 ? 5 : 6, max_m, 2); }

int tuned_small_max() { return lookup(7, 1, 32); }

}  // namespace submat
