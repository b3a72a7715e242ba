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

// Storage forms of the sweep: element type S, arithmetic type T and how the
// new deviations are rounded into S.
struct FormF64 {
  using S = double;
  static constexpr bool kStochastic = false;
};
struct FormF32 {
  using S = float;
  static constexpr bool kStochastic = false;
};
struct FormF16 {
  using S = _Float16;
  static constexpr bool kStochastic = false;
};
// FP16 with stochastic rounding: h rounds up or down to its two neighbouring
// half values with probabilities that make the rounding unbiased,
// E[h] = d * 2^8.  With round-to-nearest, a steady state rounds the same way
// at every step and the rounding acts as a constant forcing whose effect
// accumulates; unbiased rounding turns it into zero-mean noise.  The random
// numbers come from a counter-based hash of (step, node, population), so a
// lattice's results are reproducible and do not depend on the launch.
struct FormF16SR {
  using S = _Float16;
  static constexpr bool kStochastic = true;
};

// murmur3 finalizer: a bijective 32-bit mixing function.
__host__ __device__ __forceinline__ unsigned fmix32(unsigned h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Key of time step t for the stochastic rounding.
__host__ __device__ __forceinline__ unsigned step_key(unsigned t) { return fmix32(t * 0x9e3779b1u + 0x7f4a7c15u); }

// d * 2^8 rounded stochastically to half precision; r: 32 random bits.
// gfx950's conversion with stochastic rounding adds the top 13 bits of r
// below the half-precision cut of the float before truncating (for a normal
// float a = e<<23 | m that is ((a - 0x38000000) + (r >> 19)) >> 13), so it
// rounds up with probability (m mod 2^13) / 2^13 and E[h] = d * 2^8; a carry
// out of the mantissa moves to the next binade, and half subnormals are
// rounded the same way.
__device__ __forceinline__ _Float16 encode_half_sr(float d, unsigned r) {
  typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
  // The conversion writes the low half and keeps the high half of its
  // destination; only the low half is used, so the destination starts as
  // the random word itself rather than a zeroed register.
  half2_t v = __builtin_bit_cast(half2_t, r);
  v = __builtin_amdgcn_cvt_sr_f16_f32(v, d * 256.0f, r, false);
  return v[0];
}

template <class F>
__device__ __forceinline__ typename F::S encode_form(typename Codec<typename F::S>::T v, unsigned r) {
  if constexpr (F::kStochastic)
    return encode_half_sr(v, r);
  else
    return Codec<typename F::S>::encode(v);
}

// Pointer into global memory.  Kernels whose buffer addresses come from
// memory (not from kernel arguments) use it so that the compiler emits global
// rather than flat loads and stores.
template <class S>
using global_ptr = __attribute__((address_space(1))) S *;

template <class S, bool NT, class P>
__device__ __forceinline__ void store_elem(P p, S v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Maximum over the 64 lanes of a wave (every lane active).
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// Convergence measure of one node: the velocity of the stored state,
// u = sum_k c_k d_k / (1 + sum_k d_k) in double from the stored deviations
// (eq_vel), against the snapshot of the previous check.  Returns
// max_a |u_a - snap_a| / u_ref (+inf for NaN) and replaces the snapshot.
// snap: [3][N] floats; n: the node's index x + nx (y + ny z).
template <class S, class SnapP>
__device__ __forceinline__ float velocity_change(const S (&raw)[19], SnapP snap, size_t N, unsigned n,
                                                 double inv_uref) {
  double dr = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const double v = double(Codec<S>::decode(raw[k]));
    dr += v;
    if (cx(k)) j[0] += double(cx(k)) * v;
    if (cy(k)) j[1] += double(cy(k)) * v;
    if (cz(k)) j[2] += double(cz(k)) * v;
  }
  const double ir = 1.0 / (1.0 + dr);
  float dmax = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = j[a] * ir;
    const auto sp = snap + size_t(a) * N + n;
    const float du = float(fabs(u - double(*sp)) * inv_uref);
    dmax = (du != du) ? INFINITY : fmaxf(dmax, du);
    *sp = float(u);
  }
  return dmax;
}

// Where the sweep that ends a chunk of the batch runtime takes the
// convergence measure of the state it writes.
struct DeltaArgs {
  global_ptr<float> snap;  // [3][N] velocity of the previous check
  size_t N;
  double inv_uref;  // 1 / velocity scale
};

// Logical block index.  The dispatcher hands workgroups to the 8 XCDs
// round-robin (workgroup b runs on XCD b % 8).  remap 1 (slabs): logical
// blocks [q*i, q*(i+1)) all run on XCD i, so each XCD sweeps one contiguous
// eighth of the lattice.  remap 2 (rows): the g segments of one x-row run one
// after another on one XCD and rows are dealt to the XCDs in turn, so the
// x-shift overlap of a row's segments stays in one L2 while the whole chip
// sweeps one compact front (with g = 1 this is the dispatch order).  Blocks
// past the last whole round keep their index.
__host__ __device__ __forceinline__ unsigned logical_block(unsigned b, unsigned nblocks, int remap, unsigned g) {
  if (remap == 1) {
    const unsigned q = nblocks >> 3;
    if (b >= (q << 3)) return b;
    return (b & 7u) * q + (b >> 3);
  }
  if (remap == 2 && g > 1) {
    const unsigned round = 8u * g;
    if (b >= nblocks / round * round) return b;
    const unsigned j = b >> 3;
    return ((j / g) * 8u + (b & 7u)) * g + j % g;
  }
  return b;
}

// Lattice extent for the gather, and the distance in elements between the
// starts of consecutive x-rows (nx in the population-major layout, 19 nx in
// the row-major one).
struct NodeGeom {
  unsigned nx, ny, nz;
  size_t row_stride;
};

// Memory access of one population buffer pair, in elements: load_at(k,
// row, x) reads element x of population k in the x-row that starts at
// element `row` (row index times NodeGeom::row_stride) of the source;
// store_at writes the destination likewise.
//
// PtrAccess: plain pointers (kernel arguments, any size).  pop_stride is the
// distance between populations of one row: P in the population-major
// layout, nx in the row-major one.
template <class S, bool NT>
struct PtrAccess {
  const S *__restrict__ src;
  S *__restrict__ dst;
  size_t pop_stride;
  // Element x of the row that starts at element `row` of population k.  For
  // 2-byte storage, with the row uniform over the wave, the address is a
  // scalar 64-bit base plus a 32-bit lane byte offset (x * 2 < 2^32), so the
  // loads need no 64-bit vector arithmetic (the FP16 forms ran 1-2% faster
  // so).  The wider forms keep the 64-bit vector address: they compute in
  // double, already spill scalar registers, and measured 0.3% slower with
  // the scalar bases.
  __device__ __forceinline__ S load_at(int k, size_t row, unsigned x) const {
    if constexpr (sizeof(S) == 2) {
      const char *base = reinterpret_cast<const char *>(src + (size_t(k) * pop_stride + row));
      return *reinterpret_cast<const S *>(base + x * unsigned(sizeof(S)));
    } else {
      return src[size_t(k) * pop_stride + (row + x)];
    }
  }
  __device__ __forceinline__ void store_at(int k, size_t row, unsigned x, S v) const {
    if constexpr (sizeof(S) == 2) {
      char *base = reinterpret_cast<char *>(dst + (size_t(k) * pop_stride + row));
      store_elem<S, NT>(reinterpret_cast<S *>(base + x * unsigned(sizeof(S))), v);
    } else {
      store_elem<S, NT>(dst + size_t(k) * pop_stride + (row + x), v);
    }
  }
};

// BufAccess: buffer loads and stores through one resource descriptor per
// buffer, with the population's start as a scalar offset (for buffers below
// 4 GiB).  Used where the buffer addresses come from memory: the scalar base
// plus one 32-bit lane offset per access keeps register pressure low, where
// 19 + 19 64-bit population bases would not fit in scalar registers.
template <class S>
__device__ __forceinline__ S buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(S) == 8)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
  else if constexpr (sizeof(S) == 4)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, int(voff), int(soff), 0));
}

template <class S>
__device__ __forceinline__ void buf_store_nt(S v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  constexpr int kNonTemporal = 2;  // cache-policy bit "nt" (gfx94x/gfx950)
  if constexpr (sizeof(S) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          int(voff), int(soff), kNonTemporal);
  else if constexpr (sizeof(S) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(voff), int(soff), kNonTemporal);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, int(voff), int(soff),
                                          kNonTemporal);
}

// Descriptor of a raw buffer (stride 0) of `bytes` bytes at p; the last word
// holds the gfx9-family data-format bits for untyped dword access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), short(0), int(bytes), 0x00020000);
}

template <class S>
struct BufAccess {
  __amdgpu_buffer_rsrc_t src, dst;
  unsigned pop_bytes;  // population stride in bytes (PopLayout::pop_stride * sizeof(S))
  unsigned oob;        // a lane offset past the descriptors' range (their size in bytes)
  __device__ __forceinline__ S load(int k, unsigned off) const {
    return buf_load<S>(src, off * unsigned(sizeof(S)), unsigned(k) * pop_bytes);
  }
  __device__ __forceinline__ void store(int k, unsigned n, S v) const {
    buf_store_nt<S>(v, dst, n * unsigned(sizeof(S)), unsigned(k) * pop_bytes);
  }
  // Rows here are population-major (row < 2^32: buffers below 4 GiB).
  __device__ __forceinline__ S load_at(int k, size_t row, unsigned x) const { return load(k, unsigned(row) + x); }
  // As load_at, but where the value is not needed (skip) the lane's offset is
  // moved past the buffer's range: the load returns zero and reads no memory.
  static constexpr bool kSkipsLoads = true;
  __device__ __forceinline__ S load_at_if(int k, size_t row, unsigned x, bool skip) const {
    const unsigned voff = skip ? oob : (unsigned(row) + x) * unsigned(sizeof(S));
    return buf_load<S>(src, voff, unsigned(k) * pop_bytes);
  }
  __device__ __forceinline__ void store_at(int k, size_t row, unsigned x, S v) const { store(k, unsigned(row) + x, v); }
};

// RowAccess: the row-major layout, where one x-row of row_stride elements
// holds all 19 populations of its nodes.  Each access goes through a
// descriptor of its row (base at the row's start, so the offsets stay small
// for any lattice size), the lane's byte offset x * sizeof(S) and the
// population's start k * pop_stride * sizeof(S) as scalar offset: no 64-bit
// vector address arithmetic and no 19 + 19 64-bit population bases in scalar
// registers (whose spills cost vector instructions).  The row must be
// uniform over the wave.
template <class S>
struct RowAccess {
  const S *src;
  S *dst;
  unsigned pop_bytes, row_bytes;  // pop_stride and row_stride in bytes (row_bytes < 2^31)
  __device__ __forceinline__ S load_at(int k, size_t row, unsigned x) const {
    return buf_load<S>(raw_buffer(src + row, row_bytes), x * unsigned(sizeof(S)), unsigned(k) * pop_bytes);
  }
  __device__ __forceinline__ void store_at(int k, size_t row, unsigned x, S v) const {
    buf_store_nt<S>(v, raw_buffer(dst + row, row_bytes), x * unsigned(sizeof(S)), unsigned(k) * pop_bytes);
  }
};

// Whether an access type can skip a load whose value is not needed
// (load_at_if); the others take the plain gather.
template <class Access, class = void>
struct SkipsLoads {
  static constexpr bool value = false;
};
template <class Access>
struct SkipsLoads<Access, decltype(void(Access::kSkipsLoads))> {
  static constexpr bool value = Access::kSkipsLoads;
};
template <class Access>
__host__ __device__ constexpr bool skips_loads() { return SkipsLoads<Access>::value; }

// Optional per-node data of the extended sweep: solid nodes (mid-grid
// bounce-back, Sec. III) and per-node velocities of velocity faces.
struct NodeExt {
  const unsigned *solid;       // [N] solid words (solid_word), or nullptr
  const double *face_v[6];     // [n_face][3] per face, or nullptr; face node
                               // order: x faces y + ny z, y faces x + nx z,
                               // z faces x + nx y
  const unsigned *code;        // [N] complex-geometry node codes, or nullptr
};

// Solid word of a node of a lattice with a solid mask (built on the host):
// bit k (k < 18) set when the source of population k, the node at -c_k
// (periodic wrap), is solid; bit 18 set when the node itself is solid.  One
// 4-byte read per node instead of the flags of its 19 sources.
constexpr unsigned kSolidSelfBit = 18u;

// Complex-geometry node code (built on the host from the node types):
// bits 0-17 the unknown populations U, bits 18-23 the wall planes as a face
// mask m (bit f: a wall with the inward normal of face f), bits 24-26 the
// rule kind.
constexpr unsigned kGeoFluid = 0u, kGeoSolid = 1u, kGeoPlaneEdgeCorner = 2u, kGeoConvexEdge = 3u, kGeoGeneral = 4u;
__host__ __device__ constexpr unsigned geo_code(unsigned kind, unsigned m, unsigned U) {
  return (kind << 24) | (m << 18) | U;
}

// One node update: pull streaming (periodic wrap on every axis; sources
// beyond a bounded face land on in-bounds values that the boundary rule then
// overwrites), boundary rule for the face mask, BGK, store.  EXT: the node
// may be solid (its populations are copied through), a population whose
// source is a solid node is bounced back (the node's own opposite
// population of the previous step), and a face node may take its velocity
// from a per-node field.
//
// DELTA: the node's convergence measure of the state it stores
// (velocity_change, with dl) is folded into *dmax.
template <class F, bool COPY, bool EXT, class T, class Access, bool DELTA = false>
__device__ __forceinline__ void update_node(const Access &mem, const NodeGeom &g, int x, int y, int z,
                                            const NodeParams<T> &p, unsigned key, const NodeExt &ext,
                                            const DeltaArgs &dl = DeltaArgs{}, float *dmax = nullptr) {
  const unsigned bc_mask = p.bc_mask;
  using S = typename F::S;
  const unsigned nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned ym = y == 0 ? ny - 1 : unsigned(y) - 1, yp = unsigned(y) == ny - 1 ? 0 : unsigned(y) + 1;
  const unsigned zm = z == 0 ? nz - 1 : unsigned(z) - 1, zp = unsigned(z) == nz - 1 ? 0 : unsigned(z) + 1;
  const unsigned xm = x == 0 ? nx - 1 : unsigned(x) - 1, xp = unsigned(x) == nx - 1 ? 0 : unsigned(x) + 1;
  // index c+1 -> coordinate - c
  const unsigned yy[3] = {yp, unsigned(y), ym};
  const unsigned zz[3] = {zp, unsigned(z), zm};
  const unsigned xs[3] = {xp, unsigned(x), xm};
  S raw[19];
  const unsigned n = (unsigned(z) * ny + unsigned(y)) * nx + unsigned(x);
  const size_t rs = g.row_stride;
  const size_t row = size_t(unsigned(z) * ny + unsigned(y)) * rs;  // uniform when y and z are
  bool solid_node = false;
  unsigned gcode = 0u, sword = 0u;
  if constexpr (EXT) {
    if (ext.solid) {
      sword = ext.solid[n];
      solid_node = (sword >> kSolidSelfBit) & 1u;
    }
    if (ext.code) {
      gcode = ext.code[n];
      solid_node = (gcode >> 24) == kGeoSolid;
    }
  }
  if (EXT && solid_node) {
    // a solid node (or solid interior of a geometry) keeps its populations
#pragma unroll
    for (int k = 0; k < 19; ++k) raw[k] = mem.load_at(k, row, unsigned(x));
  } else if (EXT && ext.solid) {
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const unsigned srow = yy[cy(k) + 1] + ny * zz[cz(k) + 1];
      // solid source: the node's own opposite population (mid-grid bounce-back)
      const bool own = k != 18 && ((sword >> k) & 1u);
      raw[k] = mem.load_at(own ? opp(k) : k, own ? row : size_t(srow) * rs, own ? unsigned(x) : xs[cx(k) + 1]);
    }
  } else {
    // A population entering from beyond a bounded face is unknown: the
    // boundary rule replaces it without reading it, so an access that can
    // skip a load cheaply does (the batch sweep's buffer loads; with rows of
    // a few dozen nodes the wrapped source of a face node lies in a cache
    // line that another wave fetches again).
    if constexpr (skips_loads<Access>()) {
      const bool fx0 = (bc_mask & 1u) && x == 0, fx1 = (bc_mask & 2u) && unsigned(x) == nx - 1;
      const bool fy0 = (bc_mask & 4u) && y == 0, fy1 = (bc_mask & 8u) && unsigned(y) == ny - 1;
      const bool fz0 = (bc_mask & 16u) && z == 0, fz1 = (bc_mask & 32u) && unsigned(z) == nz - 1;
#pragma unroll
      for (int k = 0; k < 19; ++k) {
        const bool unk = (cx(k) > 0 && fx0) || (cx(k) < 0 && fx1) || (cy(k) > 0 && fy0) ||
                         (cy(k) < 0 && fy1) || (cz(k) > 0 && fz0) || (cz(k) < 0 && fz1);
        raw[k] = mem.load_at_if(k, size_t(yy[cy(k) + 1] + ny * zz[cz(k) + 1]) * rs, xs[cx(k) + 1], unk);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 19; ++k)
        raw[k] = mem.load_at(k, size_t(yy[cy(k) + 1] + ny * zz[cz(k) + 1]) * rs, xs[cx(k) + 1]);
    }
  }
  if (!COPY && !solid_node) {
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
    if constexpr (EXT) {
      // Complex geometry: walls at rest, rule from the node code.
      const unsigned kind = gcode >> 24;
      if (kind == kGeoPlaneEdgeCorner) {
        boundary_rule<T>(f, (gcode >> 18) & 63u, p, 0u, T(0), T(0), T(0), T(1));
      } else if (kind == kGeoConvexEdge) {
        convex_edge_rule<T>(f, gcode & 0x3ffffu);
      } else if (kind == kGeoGeneral) {
        general_wall_rule<T>(f, gcode & 0x3ffffu);
      }
    }
    if (!EXT && m) box_boundary_rule<T>(f, m, p);
    if (EXT && m) {
      T vx, vy, vz, r0;
      face_values<T>(m, p, vx, vy, vz, r0);
      const double *fld = nullptr;
      unsigned idx = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b)
        if (m == (1u << b)) {
          fld = ext.face_v[b];
          idx = b < 2 ? unsigned(y) + ny * unsigned(z) : (b < 4 ? unsigned(x) + nx * unsigned(z) : unsigned(x) + nx * unsigned(y));
        }
      if (fld) {
        vx = T(fld[3 * idx]);
        vy = T(fld[3 * idx + 1]);
        vz = T(fld[3 * idx + 2]);
      }
      boundary_rule<T>(f, m, p, p.p_mask, vx, vy, vz, r0);
    }
    bgk_collide<T>(f, p.omega, p.tau_f);
    // Random words of the stochastic rounding: a hash of (node, step), then
    // a golden-ratio Weyl sequence over the populations (each word uniform;
    // only its top 13 bits are used).
    const unsigned r0 = F::kStochastic ? fmix32(n * 0x9e3779b1u + key) : 0u;
#pragma unroll
    for (int k = 0; k < 19; ++k) raw[k] = encode_form<F>(f[k], r0 + unsigned(k + 1) * 0x9e3779b9u);
  }
#pragma unroll
  for (int k = 0; k < 19; ++k) mem.store_at(k, row, unsigned(x), raw[k]);
  if constexpr (DELTA) *dmax = fmaxf(*dmax, velocity_change<S>(raw, dl.snap, dl.N, n, dl.inv_uref));
}

}  // namespace lbm
