// node_update.hpp -- the per-node update shared by the single-lattice sweep
// and the multi-lattice (batch) sweep: pull gather of the 19 populations,
// boundary rule, BGK collision, store.  Both kernels call the same function,
// so a lattice gives bit-identical results whichever kernel advances it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "d3q19.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Storage codecs: population element type S, arithmetic type T.  The stored
// quantity is the deviation d_k = f_k - w_k from the rest state (w_k: lattice
// weight); the FP16 form stores it scaled, h = RNE(d * 2^8), d = h * 2^-8
// (exact scaling).
// ---------------------------------------------------------------------------
template <class S>
struct Codec;

template <>
struct Codec<double> {
  using T = double;
  static __device__ __forceinline__ T decode(double s) { return s; }
  static __device__ __forceinline__ double encode(T v) { return v; }
};

// FP32 storage is updated in double: the per-step rounding of the arithmetic
// then stays below the rounding of the stored deviations, so the steady state
// of the FP32 form is set by its storage alone.  On gfx950 a double FMA costs
// the same issue slot as an unpacked float FMA and the sweep is HBM-bound.
template <>
struct Codec<float> {
  using T = double;
  static __device__ __forceinline__ T decode(float s) { return double(s); }
  static __device__ __forceinline__ float encode(T v) { return float(v); }
};

template <>
struct Codec<_Float16> {
  using T = float;
  static __device__ __forceinline__ T decode(_Float16 s) { return static_cast<float>(s) * 0.00390625f; }
  static __device__ __forceinline__ _Float16 encode(T v) { return static_cast<_Float16>(v * 256.0f); }
};

template <class S, bool NT>
__device__ __forceinline__ void store_elem(S *p, S v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Logical block index.  The dispatcher hands workgroups to the 8 XCDs
// round-robin (workgroup b runs on XCD b % 8); with the remap, logical blocks
// [q*i, q*(i+1)) all run on XCD i, so neighbouring x-rows share one L2.
__device__ __forceinline__ unsigned logical_block(unsigned b, unsigned nblocks, int remap) {
  if (!remap) return b;
  const unsigned q = nblocks >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7u) * q + (b >> 3);
}

// Lattice extent for the gather.
struct NodeGeom {
  unsigned nx, ny, nz;
  size_t N;
};

// One node update: pull streaming (periodic wrap on every axis; sources
// beyond a bounded face land on in-bounds values that the boundary rule then
// overwrites), boundary rule for the face mask, BGK, store.
template <class S, bool NT, bool COPY, class T>
__device__ __forceinline__ void update_node(const S *__restrict__ src, S *__restrict__ dst, const NodeGeom &g,
                                            int x, int y, int z, unsigned bc_mask, T omega, const FaceVel<T> &fv) {
  const unsigned nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned ym = y == 0 ? ny - 1 : unsigned(y) - 1, yp = unsigned(y) == ny - 1 ? 0 : unsigned(y) + 1;
  const unsigned zm = z == 0 ? nz - 1 : unsigned(z) - 1, zp = unsigned(z) == nz - 1 ? 0 : unsigned(z) + 1;
  const unsigned xm = x == 0 ? nx - 1 : unsigned(x) - 1, xp = unsigned(x) == nx - 1 ? 0 : unsigned(x) + 1;
  // index c+1 -> coordinate - c
  const unsigned yy[3] = {yp, unsigned(y), ym};
  const unsigned zz[3] = {zp, unsigned(z), zm};
  const unsigned xs[3] = {xp, unsigned(x), xm};
  S raw[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const unsigned off = (yy[cy(k) + 1] + ny * zz[cz(k) + 1]) * nx + xs[cx(k) + 1];
    raw[k] = src[size_t(k) * g.N + off];
  }
  if constexpr (!COPY) {
    T f[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) f[k] = Codec<S>::decode(raw[k]);
    unsigned m = 0;
    if (x == 0) m |= bc_mask & 1u;
    if (unsigned(x) == nx - 1) m |= bc_mask & 2u;
    if (y == 0) m |= bc_mask & 4u;
    if (unsigned(y) == ny - 1) m |= bc_mask & 8u;
    if (z == 0) m |= bc_mask & 16u;
    if (unsigned(z) == nz - 1) m |= bc_mask & 32u;
    if (m) boundary_rule<T>(f, m, fv);
    bgk_collide<T>(f, omega);
#pragma unroll
    for (int k = 0; k < 19; ++k) raw[k] = Codec<S>::encode(f[k]);
  }
  const size_t n = (size_t(z) * ny + unsigned(y)) * nx + unsigned(x);
#pragma unroll
  for (int k = 0; k < 19; ++k) store_elem<S, NT>(dst + size_t(k) * g.N + n, raw[k]);
}

}  // namespace lbm
