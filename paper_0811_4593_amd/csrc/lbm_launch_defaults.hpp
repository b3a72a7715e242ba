// lbm_launch_defaults.hpp -- host-side launch defaults shared by the
// single-lattice C-ABI layer and the batch runtime (not part of the ABI).
#pragma once

namespace lbm {

// Default block width of the sweep for rows of nx nodes: the widest of 256,
// 128 and 64 threads whose row segments leave at most 1/16 of the lanes
// idle, else the one that leaves the fewest (a 300-node row takes 64-thread
// blocks: 20 idle lanes in 320 instead of 212 in 512).
inline int default_block_x(int nx) {
  int best = 0;
  long best_lanes = 0;
  for (int bx : {256, 128, 64}) {
    const long lanes = (long(nx) + bx - 1) / bx * bx;
    if (16 * (lanes - nx) <= lanes) return bx;
    if (best == 0 || lanes < best_lanes) {
      best = bx;
      best_lanes = lanes;
    }
  }
  return best;
}

}  // namespace lbm
