// Partitioned low-rank trace blocks (internal to libpolar).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <vector>

#include "polar_kernels.h"

namespace polar {

constexpr int kPlrMaxRank = 64;

// One leaf of a compressed block: rows [r0, r0+m) x columns [c0, c0+n).
// k >= 0: low rank, U (m x k, row-major) at offU and V (k x n, row-major) at
// offV of the block's data; k < 0: dense, D (m x n, row-major) at offU.
struct PlrLeafDev {
  int32_t r0, c0, m, n, k, pad;
  int64_t offU, offV;
};

// A compressed block as the apply kernel sees it (Job::M points at one).
struct PlrBlockDev {
  int32_t nleaves, ntile;
  const PlrLeafDev* leaves;
  const int32_t* tile_ptr;   // ntile + 1 offsets into tile_leaf
  const int32_t* tile_leaf;  // leaves intersecting each 64-row tile
  const double2* data;
};

struct PlrSet {
  int n = 0;
  PlrLeafDev* d_leaves = nullptr;
  int32_t* d_ptr = nullptr;
  int32_t* d_list = nullptr;
  double2* d_data = nullptr;
  PlrBlockDev* d_blocks = nullptr;
  size_t data_entries = 0, nleaves_total = 0;
  std::vector<size_t> stored;  // complex entries stored per block
  std::vector<int> nleaves;    // leaves per block

  // Compress the nb row-major n x n blocks at `blocks` (device memory) on the
  // GPU, on stream st; the result stays in device memory.
  hipError_t build(const double2* blocks, int nb, int n, int rmax, double eps, hipStream_t st);
  // Write block b back as a dense row-major n x n matrix (device `out`).
  hipError_t expand(int b, double2* out, hipStream_t st) const;
  size_t stored_entries(int b) const;
  // Write the compressed blocks (leaves, tile lists, data) as records to fp /
  // read them back into fresh device memory (false on an I/O or HIP error).
  bool save(FILE* fp) const;
  bool load(FILE* fp);
  // Take over the compressed blocks of `o` (same block count) while keeping
  // this set's block-descriptor array, so job terms that point at block(b)
  // stay valid; o is left empty.
  hipError_t adopt(PlrSet& o);
  const PlrBlockDev* block(int b) const { return d_blocks + b; }
  void release();
};

// Workspace of a PLR apply whose tiles' leaf lists are sliced over several
// workgroups: one 64-row partial per (tile, right-hand side, slice).
constexpr size_t kPlrPartEntries = (size_t)1 << 17;

// Y = P + alpha * sum_t PLR_t (Q_t + beta_t S_t) for jobs whose M_t point at PlrBlockDev.
// A launch with few tiles spreads each tile's leaves over several workgroups
// whose partial tiles go to `part` (part_n complex entries) and are summed in a
// fixed order by a second kernel; without a workspace one workgroup takes a tile.
hipError_t launch_plr_apply(const Job* jobs, int njobs, int n, int nrhs, int64_t ld, Bases bases, hipStream_t st,
                            hipEvent_t ev0, hipEvent_t ev1, double2* part = nullptr, size_t part_n = 0);

}  // namespace polar
