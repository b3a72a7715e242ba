// sweep2_box.hpp -- the two-steps-per-pass update of one workgroup's box
// (tile and z range) for lattices in the row-major layout, shared by the
// single-lattice kernel and the multi-lattice (batch) kernel, so that a
// lattice gets the same bits whichever kernel advances it.
//
// A workgroup owns a tile of 64 x BYI nodes in x and y and a range of
// z-planes, and streams along z: at each plane it first computes step 1 on
// the tile plus a one-node halo in x and y (pulling from HBM, halo nodes
// wrapped as the single sweep wraps its sources), keeps the results in LDS,
// and then computes step 2 on the tile's interior from LDS and writes it to
// HBM.  The arithmetic of every node is the single sweep's (the same
// boundary rules, collision, rounding and random words), so the state after
// the pass equals the state after two single sweeps bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "d3q19.hpp"
#include "node_update.hpp"

namespace lbm {

// Step 2 at plane z pulls population k from plane z - cz(k) of step 1.  A
// step-1 plane's populations with cz = -1 are read by step 2 in the same
// round, those with cz = 0 one round later and those with cz = +1 two
// rounds later: rings of 1, 2 and 3 planes, 38 population planes in all.
__host__ __device__ constexpr int ring_depth(int k) { return cz(k) < 0 ? 1 : (cz(k) == 0 ? 2 : 3); }
__host__ __device__ constexpr int ring_base(int k) {
  int b = 0;
  for (int j = 0; j < k; ++j) b += ring_depth(j);
  return b;
}
constexpr int kRingPlanes = ring_base(19);
static_assert(kRingPlanes == 38, "5 + 2 * 9 + 3 * 5 population planes");

template <class T>
struct Sweep2Args {
  int nx, ny, nz;
  size_t pop_stride, row_stride;  // row-major: R and 19 R
  int tiles_x, tiles_y, zc;       // tile grid (64 x BYI tiles) and planes per z range
  int xcd_remap;                  // LBM_XCD_SLABS or dispatch order
  unsigned key0, key1;            // step keys of the two steps (stochastic rounding)
  NodeParams<T> p;
};

// Faces of the bounded box the node (x, y, z) lies on (bit f: face f).
__device__ __forceinline__ unsigned box_faces(unsigned bc_mask, int x, int y, int z, int nx, int ny, int nz) {
  unsigned m = 0;
  if (x == 0) m |= bc_mask & 1u;
  if (x == nx - 1) m |= bc_mask & 2u;
  if (y == 0) m |= bc_mask & 4u;
  if (y == ny - 1) m |= bc_mask & 8u;
  if (z == 0) m |= bc_mask & 16u;
  if (z == nz - 1) m |= bc_mask & 32u;
  return m;
}

// Boundary rule and collision of one node (the plain path of update_node).
template <class T>
__device__ __forceinline__ void rule_and_collide(T (&f)[19], unsigned m, const NodeParams<T> &p) {
  if (m) box_boundary_rule<T>(f, m, p);
  bgk_collide<T>(f, p.omega, p.tau_f);
}

template <class F, int BYI>
struct Sweep2Tile {
  static constexpr int kHX = 66;                 // 64 interior columns + halo
  static constexpr int kHY = BYI + 2;            // BYI interior rows + halo
  static constexpr int kPlane = kHX * kHY;       // elements of one population plane
  static constexpr int kThreads = 64 * (BYI + 3);  // a wave per halo row and one for the halo columns
};

// Step 1 of the node (x, y, z) (wrapped lattice coordinates): pull from HBM,
// rule, collision, rounding with the first step's key; the encoded result
// goes to LDS cell `cell` of the ring planes of round p.  SrcP: a pointer to
// const S (a global-address-space pointer where the address comes from
// memory, so that the loads are global rather than flat).
// ps, rs: the lattice's population and row strides (a.pop_stride,
// a.row_stride), passed separately (see sweep2_box).
// ROWS: y is uniform over the wave, so each source row is read through a
// descriptor of its own (base at the row's start, the lane's byte offset and
// the population's start as scalar offset) rather than through 64-bit
// vector addresses.
template <class F, bool ROWS, class SrcP>
__device__ __forceinline__ void step1_node(SrcP src, typename F::S *ring, int plane_elems,
                                           const Sweep2Args<typename Codec<typename F::S>::T> &a, int x, int y, int z,
                                           int cell, int p, size_t ps, size_t rs) {
  using S = typename F::S;
  using T = typename Codec<S>::T;
  const unsigned nx = unsigned(a.nx), ny = unsigned(a.ny), nz = unsigned(a.nz);
  const unsigned ym = y == 0 ? ny - 1 : unsigned(y) - 1, yp = unsigned(y) == ny - 1 ? 0 : unsigned(y) + 1;
  const unsigned zm = z == 0 ? nz - 1 : unsigned(z) - 1, zp = unsigned(z) == nz - 1 ? 0 : unsigned(z) + 1;
  const unsigned xm = x == 0 ? nx - 1 : unsigned(x) - 1, xp = unsigned(x) == nx - 1 ? 0 : unsigned(x) + 1;
  const unsigned yy[3] = {yp, unsigned(y), ym};
  const unsigned zz[3] = {zp, unsigned(z), zm};
  const unsigned xs[3] = {xp, unsigned(x), xm};
  T f[19];
  if constexpr (ROWS) {
    // (read through readfirstlane: the compiler cannot see that the values
    // passed through the register barriers are uniform, and a descriptor it
    // takes for divergent would be built lane by lane in a loop)
    const unsigned yu = __builtin_amdgcn_readfirstlane(unsigned(y)), zu = __builtin_amdgcn_readfirstlane(unsigned(z));
    const unsigned rsu = __builtin_amdgcn_readfirstlane(unsigned(rs));
    const unsigned pb = __builtin_amdgcn_readfirstlane(unsigned(ps)) * unsigned(sizeof(S)), rb = rsu * unsigned(sizeof(S));
    const unsigned yr[3] = {yu == ny - 1 ? 0 : yu + 1, yu, yu == 0 ? ny - 1 : yu - 1};
    const unsigned zr[3] = {zu == nz - 1 ? 0 : zu + 1, zu, zu == 0 ? nz - 1 : zu - 1};
    const unsigned xo[3] = {xp * unsigned(sizeof(S)), unsigned(x) * unsigned(sizeof(S)), xm * unsigned(sizeof(S))};
    S raw[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const size_t row = size_t(yr[cy(k) + 1] + ny * zr[cz(k) + 1]) * rsu;
      raw[k] = buf_load<S>(raw_buffer((const S *)src + row, rb), xo[cx(k) + 1], unsigned(k) * pb);
    }
    // All 19 loads in flight before the first is used: without this
    // statement the compiler, short of registers, waited for each load
    // before issuing the next.
    asm volatile(""
                 : "+v"(raw[0]), "+v"(raw[1]), "+v"(raw[2]), "+v"(raw[3]), "+v"(raw[4]), "+v"(raw[5]), "+v"(raw[6]),
                   "+v"(raw[7]), "+v"(raw[8]), "+v"(raw[9]), "+v"(raw[10]), "+v"(raw[11]), "+v"(raw[12]),
                   "+v"(raw[13]), "+v"(raw[14]), "+v"(raw[15]), "+v"(raw[16]), "+v"(raw[17]), "+v"(raw[18]));
#pragma unroll
    for (int k = 0; k < 19; ++k) f[k] = Codec<S>::decode(raw[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const size_t row = size_t(yy[cy(k) + 1] + ny * zz[cz(k) + 1]) * rs;
      f[k] = Codec<S>::decode(src[size_t(k) * ps + row + xs[cx(k) + 1]]);
    }
  }
  rule_and_collide<T>(f, box_faces(a.p.bc_mask, x, y, z, a.nx, a.ny, a.nz), a.p);
  const unsigned n = (unsigned(z) * ny + unsigned(y)) * nx + unsigned(x);
  const unsigned r0 = F::kStochastic ? fmix32(n * 0x9e3779b1u + a.key0) : 0u;
  const int s2 = p & 1, s3 = p % 3;
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const int slot = ring_depth(k) == 1 ? 0 : (ring_depth(k) == 2 ? s2 : s3);
    ring[(ring_base(k) + slot) * plane_elems + cell] = encode_form<F>(f[k], r0 + unsigned(k + 1) * 0x9e3779b9u);
  }
}

// The two steps of one workgroup's box: tile (tx, ty) of 64 x BYI nodes and
// z range tz of a.zc planes, with the population ring `ring` in LDS
// (kRingPlanes * Sweep2Tile<F, BYI>::kPlane elements).  Every thread of the
// workgroup calls it (it holds barriers).  SrcP, DstP: pointers to const S
// and to S that do not alias (plain pointers from kernel arguments, or
// global-address-space pointers).
template <class F, int BYI, class SrcP, class DstP>
__device__ __forceinline__ void sweep2_box(SrcP src, DstP dst,
                                           const Sweep2Args<typename Codec<typename F::S>::T> &a, unsigned tx,
                                           unsigned ty, unsigned tz, typename F::S *ring) {
  using S = typename F::S;
  using T = typename Codec<S>::T;
  using Tile = Sweep2Tile<F, BYI>;
  constexpr int HX = Tile::kHX, HY = Tile::kHY, PLANE = Tile::kPlane;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int x0 = int(tx) * 64, y0 = int(ty) * BYI, zb = int(tz) * a.zc;
  const int ze = min(zb + a.zc, nz);
  const int w = min(64, nx - x0), hyc = min(BYI, ny - y0);  // interior columns and rows of this tile
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int lane0 = int(threadIdx.x) & 63;
  // The FP32 form reads the step-1 sources of the halo rows and writes step
  // 2 through per-row descriptors (no 64-bit vector address arithmetic:
  // 0.3-2.4% faster on 1024 x 512 x 512 and 1.8% on 512 x 256 x 256, with
  // 17% fewer vector instructions); the FP64 and FP16 forms, measured 2-5%
  // slower so, keep the pointers.
  constexpr bool kRowDescriptors = sizeof(S) == 4;

  for (int p = 0, zz = zb - 1; zz <= ze; ++p, ++zz) {
    // The lane index is passed through an empty asm statement each round, so
    // that the compiler recomputes the per-lane addresses inside the loop
    // instead of holding 2 x 19 of them in registers across it (they spilled
    // to scratch).
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    // The strides likewise (FP32 and FP16 forms): the compiler then
    // recomputes the 19 population offsets on the scalar unit each round
    // instead of holding them across the loop in spilled scalar registers,
    // which took a vector instruction per reload; 1024 x 512 x 512 FP32
    // went from 6.19 to 5.76 ms per step.  (FP64, whose tiles hold 5 rows,
    // ran 1.3% slower this way.)
    size_t ps = a.pop_stride, rs = a.row_stride;
    if constexpr (sizeof(S) < 8) asm volatile("" : "+s"(ps), "+s"(rs));
    const int z1 = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
    // Step 1 on the tile and its halo.  Waves 0..BYI+1 take the 64 interior
    // columns of halo rows 0..BYI+1 (rows past the tile's last interior row
    // + 1 idle); the last wave takes the left and right halo column of every
    // row.  Halo cells hold the wrapped nodes, as the single sweep's pull
    // reads them.
    if (wave < HY) {
      if (lane < w && wave <= hyc + 1) {
        int y = y0 + wave - 1;
        y += y < 0 ? ny : (y >= ny ? -ny : 0);
        step1_node<F, kRowDescriptors, SrcP>(src, ring, PLANE, a, x0 + lane, y, z1, wave * HX + lane + 1, p, ps,
                                             rs);
      }
    } else {
      const int hy = lane >> 1, right = lane & 1;
      if (lane < 2 * HY && hy <= hyc + 1) {
        int y = y0 + hy - 1;
        y += y < 0 ? ny : (y >= ny ? -ny : 0);
        int x = right ? x0 + w : x0 - 1;
        x += x < 0 ? nx : (x >= nx ? -nx : 0);
        step1_node<F, false, SrcP>(src, ring, PLANE, a, x, y, z1, hy * HX + (right ? w + 1 : 0), p, ps, rs);
      }
    }
    __syncthreads();
    // Step 2 on the interior of plane zz - 1, from LDS.
    if (p >= 2 && wave < hyc && lane < w) {
      const int z2 = zz - 1, y2 = y0 + wave, x2 = x0 + lane;
      const int c = (wave + 1) * HX + lane + 1;  // the node's own cell
      const int q0 = (p + 1) & 1, q1 = (p + 1) % 3;  // ring slots of rounds p - 1 (cz = 0) and p - 2 (cz = +1)
      T f[19];
#pragma unroll
      for (int k = 0; k < 19; ++k) {
        const int slot = ring_depth(k) == 1 ? 0 : (ring_depth(k) == 2 ? q0 : q1);
        f[k] = Codec<S>::decode(ring[(ring_base(k) + slot) * PLANE + c - cy(k) * HX - cx(k)]);
      }
      rule_and_collide<T>(f, box_faces(a.p.bc_mask, x2, y2, z2, nx, ny, nz), a.p);
      const unsigned n = (unsigned(z2) * unsigned(ny) + unsigned(y2)) * unsigned(nx) + unsigned(x2);
      const unsigned r0 = F::kStochastic ? fmix32(n * 0x9e3779b1u + a.key1) : 0u;
      const size_t row = size_t(unsigned(z2) * unsigned(ny) + unsigned(y2)) * rs;
      if constexpr (kRowDescriptors) {
        // the row is uniform over the wave: stores through its descriptor
        const auto out = raw_buffer((S *)dst + row, unsigned(rs) * unsigned(sizeof(S)));
        const unsigned pb = unsigned(ps) * unsigned(sizeof(S)), xo = unsigned(x2) * unsigned(sizeof(S));
#pragma unroll
        for (int k = 0; k < 19; ++k)
          buf_store_nt<S>(encode_form<F>(f[k], r0 + unsigned(k + 1) * 0x9e3779b9u), out, xo, unsigned(k) * pb);
      } else {
#pragma unroll
        for (int k = 0; k < 19; ++k)
          store_elem<S, true>(dst + size_t(k) * ps + row + unsigned(x2),
                              encode_form<F>(f[k], r0 + unsigned(k + 1) * 0x9e3779b9u));
      }
    }
    __syncthreads();
  }
}

// Interior rows per tile of each storage form.  LDS holds 38 population
// planes of 66 x (BYI + 2) elements: 147 KB for FP32 with BYI = 13 (one
// workgroup of 16 waves per compute unit; step 1 then costs 1.2 times the
// updates it feeds), 137 KB for FP64 with BYI = 5, 73 KB for FP16 with
// BYI = 13.
template <class F>
struct Sweep2Rows;
template <>
struct Sweep2Rows<FormF64> {
  static constexpr int kBYI = 5;
};
template <>
struct Sweep2Rows<FormF32> {
  static constexpr int kBYI = 13;
};
template <>
struct Sweep2Rows<FormF16> {
  static constexpr int kBYI = 13;
};
template <>
struct Sweep2Rows<FormF16SR> {
  static constexpr int kBYI = 13;
};

}  // namespace lbm
