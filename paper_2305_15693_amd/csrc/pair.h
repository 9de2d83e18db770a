// Soft-core pair repulsion on a cell list: context and the launcher the loss
// context calls when a pair term is attached to it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "fresco.h"

struct fresco_pair_ctx {
  int d = 0;
  int dtype = 0;
  long long n = 0;
  double L[3] = {1.0, 1.0, 1.0};
  double sigma = 0.0, eps = 0.0, alpha = 0.0;
  int nc[3] = {1, 1, 1};  // cells per axis (side L_a / nc_a >= sigma)
  long long ncell = 1;
  hipStream_t st = nullptr;
  std::vector<void*> allocs;
  uint32_t* key = nullptr;     // [n] cell of each point
  uint32_t* rank = nullptr;    // [n] arrival rank inside the cell
  uint32_t* count = nullptr;   // [ncell]
  uint32_t* start = nullptr;   // [ncell + 1]
  uint32_t* bsum = nullptr;    // scan block sums
  int nscan_blocks = 0;
  void* sorted = nullptr;      // [n] records (position, original index), cell order
  double* part = nullptr;      // [nblocks] FP64 energy partials
  int nblocks = 0;
  int* flag = nullptr;         // set for a non-finite position
  double* edev = nullptr;      // energy of the synchronous call
  int* fout = nullptr;         // flag of the synchronous call
  double* energy_host = nullptr;  // pinned: energy, then the flag
  // overlap replacement (allocated on first use): flags, their exclusive scan
  // (n + 1 entries, the last the count), scan block sums
  uint32_t* oflag = nullptr;
  uint32_t* orank = nullptr;
  uint32_t* obsum = nullptr;
  uint32_t* ocount_host = nullptr;  // pinned copy of the count
};

namespace fresco {

// Enqueue the pair pass on st: energy partials into pc->part (pc->nblocks of
// them, to be summed in order) and the gradient into grad (added to it when
// accumulate, else written).  weight scales the gradient.
int pair_enqueue(fresco_pair_ctx* pc, const void* pos, void* grad, bool accumulate, double weight,
                 hipStream_t st);

}  // namespace fresco
