// tune_cache.hpp -- launch shapes and the process-wide store of autotuned
// choices, with its JSON file.  Host code only (no HIP), so that it also
// builds with the host compiler alone.
#pragma once
#include <stdint.h>

#include <string>

namespace dgal {

// Launch shape of one call, chosen by the autotuner (0 = built-in default).
// grid: workgroups of a grid-stride elementwise kernel (0 => one lane per
// item); the matrix multipliers scale the persistent grids by the CU count;
// tile_rows sets the matrix tiles (tile_rows x 2048 / tile_rows pairs).
struct LaunchShape {
  int64_t grid = 0;
  int cull_mult = 0, exact_mult = 0, bwd_mult = 0;
  int tile_rows = 0;
};

inline bool operator==(const LaunchShape& x, const LaunchShape& y) {
  return x.grid == y.grid && x.cull_mult == y.cull_mult && x.exact_mult == y.exact_mult &&
         x.bwd_mult == y.bwd_mult && x.tile_rows == y.tile_rows;
}

// Whether every field is one the library can launch (the file is input).
bool shape_valid(const LaunchShape& s);

// The store: key -> (shape, milliseconds of the timed runs that chose it).
// Keys name the GPU architecture and the kind of call, e.g.
// "gfx950/matrix_fwd/K4/fixed1/z1/seg1/b13.6".  Thread-safe.
bool tune_store_get(const std::string& key, LaunchShape* out);
void tune_store_put(const std::string& key, const LaunchShape& s, double ms);
void tune_store_clear();
int64_t tune_store_size();

// Merges the entries of a JSON cache file into the store (a file entry
// replaces the store's entry of the same key).  Returns the number of entries
// read, DGAL_EIO if the file cannot be read, DGAL_EINVAL if it is not a cache
// file (then nothing is merged).
int tune_store_load(const char* path);
// Writes the whole store to `path` (a temporary file renamed over it).
// DGAL_OK or DGAL_EIO.
int tune_store_save(const char* path);
// One line per entry, "<key> grid=.. cull=.. exact=.. bwd=.. rows=.. ms=..",
// into buf (NUL-terminated, truncated to size); returns the entry count.
int tune_store_report(char* buf, int64_t size);

// The cache file named by DGAL_TUNE_CACHE, loaded once per process if it
// exists (a missing file is written after the first tuning).  Returns the
// path, or NULL when the variable is unset or empty, or names a file that
// exists but does not load as a cache (which is then never written).
const char* tune_cache_path();

}  // namespace dgal
