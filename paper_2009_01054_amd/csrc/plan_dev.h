// Device-side plan construction (internal).  The index work of a plan --
// validation and unique counts (Table 1), the sorts of the input pairs into
// stage-1 key segments, the output groupings and the stage-2 tile orders --
// runs as kernels and stable radix sorts on the plan's stream.  Every sort is
// stable, so the arrays are the ones the host construction produces.
#pragma once

#include "common.h"

namespace gvt {

// Smallest b with 2^b >= range.
inline int bits_for(int64_t range) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < range) ++b;
  return b;
}

// Scratch of one device plan build: key and value buffers and the sort's
// temporary storage, grown on demand.  Builds that share it must run on one
// stream.
struct DevScratch {
  DevMem mem;
  size_t need = 0;
};

// Per index array i < narr: the first position holding a value outside
// [0, lim[i]) (or -1), and a byte per value in [0, range[i]) set when the value
// occurs.  `nat`: with natural-order limits (nat_cols > 0), whether arrays 0/1
// and 2/3 hold the full grid in row-major order (complete data).
struct ProbeResult {
  int64_t bad[4] = {-1, -1, -1, -1};
  std::vector<uint8_t> seen[4];
  bool nat = false;
};
void dev_probe(const int32_t *const *x, const int64_t *n, const int64_t *lim, const int64_t *range,
               int narr, int64_t nat_out_cols, int64_t nat_in_cols, DevScratch &sc,
               ProbeResult &res, hipStream_t s);

// Scratch bytes each builder below needs, and growing the scratch ahead of a
// series of builds (growing it later waits for the queued ones).
size_t dev_input_sort_bytes(int64_t nkeys, int64_t nother, int64_t n);
size_t dev_group_rows_bytes(int64_t n);
size_t dev_tiles_bytes(int64_t n, int64_t nbuckets);
void dev_reserve(DevScratch &sc, size_t bytes, hipStream_t s);

// Input pairs sorted by (key, other), stable: perm[p] = input index at sorted
// position p, other[p] its other index, seg[k] the first position of key k
// (seg[nkeys] = n).
void dev_input_sort(const int32_t *key, int64_t nkeys, const int32_t *other, int64_t nother,
                    int64_t n, int32_t *perm, int32_t *other_out, int64_t *seg, DevScratch &sc,
                    hipStream_t s);

// inv[perm[p]] = p for p < n.
void dev_invert(const int32_t *perm, int64_t n, int32_t *inv, hipStream_t s);

// Output positions grouped by `row` (stable): perm[q] = output index, off[r]
// the first position of row value r (off[nrows] = n).
void dev_group_rows(const int32_t *row, int64_t nrows, int64_t n, int32_t *perm, int64_t *off,
                    DevScratch &sc, hipStream_t s);

// Stage-2 tiles (see compute_tiles): outputs keyed by (tile, group row) with
// grp / stg the grouped and staged coordinate of each output (grp from `gx`,
// stg from `sy` through `rowmap`, swapped when `swap`); `grow` lists each
// tile's group rows by descending output count (ties by row).
struct TileDims {
  int64_t ntiles, nsb, sbs, nstg_rows, rows_per_tile;
  bool swap;  // class 1: group by compact S row, stage F1 rows
};
void dev_tiles(const int32_t *gx, const int32_t *sy, const int32_t *rowmap, int64_t n,
               const TileDims &td, int32_t *perm, int32_t *yrows, int64_t *toff, int32_t *tiley,
               int32_t *tilemax, uint8_t *grow, DevScratch &sc, hipStream_t s);

}  // namespace gvt
