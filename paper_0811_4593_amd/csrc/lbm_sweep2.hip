// lbm_sweep2.hip -- two time steps per pass over HBM (temporal blocking) for
// lattices in the row-major layout.
//
// The single sweep reads and writes every population once per step, so at
// the HBM bandwidth it can do no better than a copy.  Here a workgroup owns a
// tile of 64 x BYI nodes in x and y and a range of z-planes, and streams
// along z: at each plane it first computes step 1 on the tile plus a
// one-node halo in x and y (pulling from HBM, halo nodes wrapped as the
// single sweep wraps its sources), keeps the results in LDS, and then
// computes step 2 on the tile's interior from LDS and writes it to HBM.  Per
// node and two steps it reads the 19 populations once (plus the halo, shared
// with the neighbouring tiles through L2) and writes them once: about half
// the bytes of two single sweeps.  The arithmetic of every node is the single
// sweep's (the same boundary rules, collision, rounding and random words), so
// the state after the pass equals the state after two single sweeps bit for
// bit.  The update of one workgroup's box is sweep2_box (sweep2_box.hpp),
// which the batch runtime's multi-lattice pass calls as well.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "d3q19.hpp"
#include "lbm_internal.hpp"
#include "node_update.hpp"
#include "sweep2_box.hpp"

namespace lbm {

template <class F, int BYI>
__global__ __launch_bounds__(64 * (BYI + 3)) void sweep2_kernel(
    const typename F::S *__restrict__ src, typename F::S *__restrict__ dst,
    Sweep2Args<typename Codec<typename F::S>::T> a) {
  using S = typename F::S;
  __shared__ S ring[kRingPlanes * Sweep2Tile<F, BYI>::kPlane];
  const unsigned b = logical_block(blockIdx.x, gridDim.x, a.xcd_remap, 1u);
  const unsigned tx = b % unsigned(a.tiles_x), rest = b / unsigned(a.tiles_x);
  const unsigned ty = rest % unsigned(a.tiles_y), tz = rest / unsigned(a.tiles_y);
  sweep2_box<F, BYI, const S *__restrict__, S *__restrict__>(src, dst, a, tx, ty, tz, ring);
}

template <class F, int BYI>
static hipError_t launch_sweep2_t(const SweepConfig &c, int zc, const void *src, void *dst, hipStream_t s) {
  using S = typename F::S;
  using T = typename Codec<S>::T;
  Sweep2Args<T> a;
  a.nx = c.nx;
  a.ny = c.ny;
  a.nz = c.nz;
  a.pop_stride = c.layout.pop_stride;
  a.row_stride = c.layout.row_stride;
  a.tiles_x = (c.nx + 63) / 64;
  a.tiles_y = (c.ny + BYI - 1) / BYI;
  a.zc = zc;
  a.xcd_remap = c.xcd_remap == 1 ? 1 : 0;
  a.key0 = step_key(c.step);
  a.key1 = step_key(c.step + 1u);
  a.p.bc_mask = c.bc_mask;
  a.p.p_mask = c.p_mask;
  a.p.rule_flags = c.rule_flags;
  a.p.omega = T(1.0 / c.tau);
  for (int d = 0; d < 3; ++d) a.p.tau_f[d] = T(c.tau * c.force[d]);
  for (int f = 0; f < 6; ++f) a.p.rho_p[f] = T(c.rho_p[f]);
  for (int f = 0; f < 6; ++f)
    for (int d = 0; d < 3; ++d) a.p.fv.v[f][d] = T(c.v[f][d]);
  const size_t tiles_z = (size_t(c.nz) + size_t(zc) - 1) / size_t(zc);
  const size_t nblocks = size_t(a.tiles_x) * size_t(a.tiles_y) * tiles_z;
  if (nblocks == 0 || nblocks > 0x7fffffffu) return hipErrorInvalidValue;
  sweep2_kernel<F, BYI><<<dim3(unsigned(nblocks)), dim3(Sweep2Tile<F, BYI>::kThreads), 0, s>>>(
      static_cast<const S *>(src), static_cast<S *>(dst), a);
  return hipGetLastError();
}

hipError_t launch_sweep2(const SweepConfig &c, int zc, int rows, const void *src, void *dst, hipStream_t s) {
  // row-major layout only: the tile's rows are whole rows of one population
  if (c.layout.row_stride != 19 * c.layout.pop_stride || zc < 1) return hipErrorInvalidValue;
  switch (c.storage) {
    case kStoreF64: return launch_sweep2_t<FormF64, Sweep2Rows<FormF64>::kBYI>(c, zc, src, dst, s);
    case kStoreF32:
      if (rows == 5) return launch_sweep2_t<FormF32, 5>(c, zc, src, dst, s);
      if (rows == 12) return launch_sweep2_t<FormF32, 12>(c, zc, src, dst, s);
      return launch_sweep2_t<FormF32, Sweep2Rows<FormF32>::kBYI>(c, zc, src, dst, s);
    case kStoreF16:
      if (rows == 5) return launch_sweep2_t<FormF16, 5>(c, zc, src, dst, s);
      if (rows == 12) return launch_sweep2_t<FormF16, 12>(c, zc, src, dst, s);
      return launch_sweep2_t<FormF16, Sweep2Rows<FormF16>::kBYI>(c, zc, src, dst, s);
    case kStoreF16SR:
      if (rows == 5) return launch_sweep2_t<FormF16SR, 5>(c, zc, src, dst, s);
      if (rows == 12) return launch_sweep2_t<FormF16SR, 12>(c, zc, src, dst, s);
      return launch_sweep2_t<FormF16SR, Sweep2Rows<FormF16SR>::kBYI>(c, zc, src, dst, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
