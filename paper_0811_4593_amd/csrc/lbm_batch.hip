// lbm_batch.hip -- many independent lattices on one GPU: a persistent
// multi-lattice sweep over a tile list, a device memory pool with admission by
// an HBM budget, step chunks captured in HIP graphs, a per-lattice
// convergence measure, and an autotuner for the launch shape.
//
// Every lattice is advanced by the same per-node update as the single-lattice
// sweep (node_update.hpp), so a lattice gives bit-identical results alone or
// in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <new>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"
#include "lbm_launch_defaults.hpp"
#include "node_update.hpp"
#include "sweep2_box.hpp"

namespace lbm {

// Device-side description of one resident lattice.
struct BatchLat {
  void *buf[2];    // population buffers (state in buf[0] at chunk boundaries)
  float *snap;     // [3][N] velocity at the previous convergence check
  unsigned nx, ny, nz, N;
  unsigned buf_elems;               // elements per population buffer
  unsigned pop_stride, row_stride;  // PopLayout of the buffers, in elements
  unsigned slot_row;                // tile slots per x-row: nx, or the padded row pitch
  unsigned bc_mask;
  unsigned p_mask;     // pressure faces
  unsigned step_base;  // steps taken before the current launch sequence
  double omega;    // 1 / tau
  double v[6][3];  // face velocities (pressure faces: tangential velocity)
  double rho_p[6]; // prescribed densities of the pressure faces
  double tau_f[3]; // tau * body force
  double inv_uref; // 1 / velocity scale of the convergence measure
};

// Inward unit normals of the faces x0, x1, y0, y1, z0, z1.
static const int kFaceNormal[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

// A contiguous range [n0, n1) of one lattice's slots: slot s is node
// x = s % slot_row of x-row s / slot_row, x >= nx a padding slot (no node).
struct BatchTile {
  int lat;
  unsigned n0, n1;
};

// Consecutive tiles that run on one XCD, one after another, when every tile
// has a workgroup of its own: the cache lines that neighbouring tiles share
// (a shifted population range starts and ends inside lines) are then fetched
// once into that XCD's L2, while the chip still sweeps the tile list as one
// compact front.  On 64 uneven ducts in FP32 the batch step took 1.305 ms
// with groups of 4, 1.307 ms in dispatch order (FETCH 1.10x the algorithmic
// reads) and 1.446 ms with one contiguous eighth of the list per XCD (FETCH
// 0.99x): the fewest re-reads do not make the fastest order.
constexpr unsigned kTileGroup = 4;

// One step of every lattice of storage form F listed in `tiles`.  With own
// (the default shape: a grid of one workgroup per entry of the tile table)
// every tile has a workgroup of its own, tiles dealt to the XCDs in groups
// of kTileGroup (logical_block); otherwise the grid's workgroups walk the
// list round-robin (persistent workgroups).  Each lane updates the nodes of slots n0 + t, n0 + t + BX, ...
// of its tile (the padding slots of a row-major lattice with padded rows stay
// idle, so that its rows' waves start on cache lines as the rows do).  `s` is
// the index of the step within the launch sequence (with the lattice's
// step_base, the step key); the step reads buf[parity] and writes the other.
//
// One workgroup per tile beat persistent workgroups by 14% on the 64 ducts
// (1.305 against 1.510 ms per step, tiles of 256 against the persistent
// walk's best, 1024 nodes and 16 workgroups per CU): a persistent workgroup
// waits on the dependent loads of each new tile's descriptor and lattice
// parameters before its first gather, where fresh workgroups start while
// others still run.
// Node-update parameters of a lattice in the arithmetic type T.
template <class T>
__device__ __forceinline__ NodeParams<T> lattice_params(const BatchLat &L) {
  NodeParams<T> prm;
  prm.bc_mask = L.bc_mask;
  prm.p_mask = L.p_mask;
  prm.rule_flags = 0u;
  prm.omega = T(L.omega);
#pragma unroll
  for (int f = 0; f < 6; ++f) prm.rho_p[f] = T(L.rho_p[f]);
#pragma unroll
  for (int d = 0; d < 3; ++d) prm.tau_f[d] = T(L.tau_f[d]);
#pragma unroll
  for (int f = 0; f < 6; ++f)
#pragma unroll
    for (int d = 0; d < 3; ++d) prm.fv.v[f][d] = T(L.v[f][d]);
  return prm;
}

//
// DELTA (one workgroup per tile only): the step ends a chunk and also takes
// the convergence measure of the state it writes; each wave's maximum goes
// to partials[tile * BX / 64 + wave] (tile_partials_kernel then combines
// them per lattice).
template <class F, int BX, bool DELTA, bool OWN>
__global__ __launch_bounds__(BX) void batch_sweep_kernel(const BatchLat *__restrict__ lats,
                                                         const BatchTile *__restrict__ tiles,
                                                         const int *__restrict__ ntiles, int s, int parity,
                                                         float *__restrict__ partials) {
  static_assert(OWN || !DELTA, "the measure needs a workgroup per tile");
  using S = typename F::S;
  using T = typename Codec<S>::T;
  auto step_tile = [&](int t, const BatchTile &tile) {
    const BatchLat &L = lats[tile.lat];
    const NodeGeom g{L.nx, L.ny, L.nz, size_t(L.row_stride)};
    const unsigned buf_bytes = L.buf_elems * unsigned(sizeof(S));
    const BufAccess<S> mem{raw_buffer(L.buf[parity], buf_bytes), raw_buffer(L.buf[parity ^ 1], buf_bytes),
                           L.pop_stride * unsigned(sizeof(S)), buf_bytes};
    const NodeParams<T> prm = lattice_params<T>(L);
    const unsigned key = step_key(L.step_base + unsigned(s));
    // Coordinates of the lane's first slot, then advanced by BX slots per
    // iteration with carries (one division per tile instead of two per node).
    const unsigned sr = L.slot_row;
    unsigned n = tile.n0 + threadIdx.x;
    unsigned r = n / sr;
    unsigned x = n - r * sr;
    unsigned z = r / g.ny;
    unsigned y = r - z * g.ny;
    const unsigned rows = unsigned(BX) / sr;  // uniform
    const unsigned dx = unsigned(BX) - rows * sr;
    const unsigned dz = rows / g.ny;
    const unsigned dy = rows - dz * g.ny;
    DeltaArgs dl{};
    float dmax = 0.0f;
    if constexpr (DELTA) dl = DeltaArgs{(global_ptr<float>)(L.snap), size_t(L.N), L.inv_uref};
    for (; n < tile.n1; n += BX) {
      if (x < g.nx)
        update_node<F, false, false, T, BufAccess<S>, DELTA>(mem, g, int(x), int(y), int(z), prm, key, NodeExt{}, dl,
                                                             &dmax);
      x += dx;
      const unsigned cxr = x >= sr;
      x -= cxr ? sr : 0u;
      y += dy + cxr;
      const unsigned cyr = y >= g.ny;
      y -= cyr ? g.ny : 0u;
      z += dz + cyr;
    }
    if constexpr (DELTA) {
      dmax = wave_max(dmax);
      if ((threadIdx.x & 63) == 0) partials[size_t(t) * (BX / 64) + (threadIdx.x >> 6)] = dmax;
    }
  };
  if constexpr (OWN) {
    // One workgroup per entry of the tile table (the grid is its capacity):
    // the tile follows from the block index alone, so its record is loaded
    // beside the tile count rather than after it, and workgroups past the
    // count exit.
    const int t = int(logical_block(blockIdx.x, gridDim.x, 2, kTileGroup));
    BatchTile tile = tiles[t];
    int nt = *ntiles;
    // both loads in flight before either is waited for (the compiler would
    // otherwise load the tile only after the count check)
    asm volatile("" : "+s"(tile.lat), "+s"(tile.n0), "+s"(tile.n1), "+s"(nt));
    if (t < nt) step_tile(t, tile);
  } else {
    const int nt = *ntiles;
    for (int b = blockIdx.x; b < nt; b += gridDim.x) step_tile(b, tiles[b]);
  }
}

// Convergence measure, per lattice: max over nodes and components of
// |u(t) - u(t_prev)| / u_ref (u from the stored state, eq_vel), then the
// snapshot is replaced by u(t).  Maxima are combined with an atomic max on
// the bit pattern of non-negative floats: order-independent, so the stop step
// of every lattice is deterministic.  NaN counts as +inf.  The sweep that
// ends a chunk takes the measure of the state it writes (update_node with
// DELTA); with two steps per pass this kernel takes it afterwards.

// The workgroup's maximum of v into delta_bits[lat] (every thread calls it).
__device__ __forceinline__ void flush_max(float v, unsigned *delta_bits, int lat, float *lds) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(lds[0], lds[1]), fmaxf(lds[2], lds[3]));
    atomicMax(delta_bits + lat, __float_as_uint(m));
  }
  __syncthreads();
}

// Each persistent workgroup takes one contiguous share of the tile list and
// keeps each lane's maximum across the consecutive tiles of one lattice,
// flushing it with one atomic when the lattice changes: a launch issues
// about one atomic per workgroup and lattice instead of one per tile (a
// 256^3 lattice has 65536 tiles of 256 nodes; their atomics on one address
// serialised the launch), and the next tile's nodes follow the last one's
// in memory.
template <class S>
__global__ __launch_bounds__(256) void batch_delta_kernel(const BatchLat *__restrict__ lats,
                                                          const BatchTile *__restrict__ tiles,
                                                          const int *__restrict__ ntiles,
                                                          unsigned *__restrict__ delta_bits) {
  __shared__ float lds[4];
  const int nt = *ntiles;
  const int t0 = int((long long)nt * blockIdx.x / gridDim.x);
  const int t1 = int((long long)nt * (blockIdx.x + 1) / gridDim.x);
  int cur = -1;  // lattice of the running maximum (uniform over the workgroup)
  float dmax = 0.0f;
  for (int t = t0; t < t1; ++t) {
    const BatchTile tile = tiles[t];
    if (tile.lat != cur) {
      if (cur >= 0) flush_max(dmax, delta_bits, cur, lds);
      cur = tile.lat;
      dmax = 0.0f;
    }
    const BatchLat &L = lats[tile.lat];
    const global_ptr<const S> f = (global_ptr<const S>)(L.buf[0]);
    const global_ptr<float> snap = (global_ptr<float>)(L.snap);
    for (unsigned sl = tile.n0 + threadIdx.x; sl < tile.n1; sl += 256) {
      const unsigned r = sl / L.slot_row, x = sl - r * L.slot_row;
      if (x >= L.nx) continue;  // padding slot
      S raw[19];
      const size_t at = size_t(r) * L.row_stride + x;
#pragma unroll
      for (int k = 0; k < 19; ++k) raw[k] = f[at + size_t(k) * L.pop_stride];
      dmax = fmaxf(dmax, velocity_change<S>(raw, snap, L.N, r * L.nx + x, L.inv_uref));
    }
  }
  if (cur >= 0) flush_max(dmax, delta_bits, cur, lds);
}

// The per-wave maxima of a chunk's last batch sweep (DELTA), per lattice:
// as batch_delta_kernel, each persistent workgroup takes a contiguous share
// of the tile list and flushes once per lattice; it reads `waves` partials
// per tile instead of the state.  A round covers 256 / waves tiles of one
// lattice (the tiles of a lattice are contiguous, so a round whose first
// and last tile share a lattice lies in it); a round across a lattice's
// end goes tile by tile.
__global__ __launch_bounds__(256) void tile_partials_kernel(const BatchTile *__restrict__ tiles,
                                                            const int *__restrict__ ntiles,
                                                            const float *__restrict__ partials, int waves,
                                                            unsigned *__restrict__ delta_bits) {
  __shared__ float lds[4];
  const int nt = *ntiles;
  const int t0 = int((long long)nt * blockIdx.x / gridDim.x);
  const int t1 = int((long long)nt * (blockIdx.x + 1) / gridDim.x);
  const int per_round = 256 / waves, tid = int(threadIdx.x);
  int cur = -1;  // lattice of the running maximum (uniform over the workgroup)
  float dmax = 0.0f;
  for (int base = t0; base < t1; base += per_round) {
    const int last = min(base + per_round, t1) - 1;
    const int la = tiles[base].lat, lb = tiles[last].lat;
    if (la == lb) {
      if (la != cur) {
        if (cur >= 0) flush_max(dmax, delta_bits, cur, lds);
        cur = la;
        dmax = 0.0f;
      }
      const int t = base + tid / waves;
      if (t <= last) dmax = fmaxf(dmax, partials[size_t(t) * waves + tid % waves]);
    } else {
      for (int u = base; u <= last; ++u) {
        const int l = tiles[u].lat;
        if (l != cur) {
          if (cur >= 0) flush_max(dmax, delta_bits, cur, lds);
          cur = l;
          dmax = 0.0f;
        }
        if (tid < waves) dmax = fmaxf(dmax, partials[size_t(u) * waves + tid]);
      }
    }
  }
  if (cur >= 0) flush_max(dmax, delta_bits, cur, lds);
}

__global__ void fill_float_kernel(float *__restrict__ p, size_t n, float v) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One box of the multi-lattice two-step pass: tile (tx, ty) of 64 x BYI
// nodes and z range tz of lattice `lat` (row-major).
struct BatchBox {
  int lat;
  unsigned tx, ty, tz;
};

// Steps s and s + 1 of every lattice of storage form F listed in `boxes`,
// one workgroup per box (workgroups past the box count exit at once): the
// single-lattice two-step pass's box update (sweep2_box) with the lattice's
// parameters from its descriptor, reading buf[parity] and writing the other
// buffer, so that each lattice gets the bits of two single sweeps.  remap:
// the box list's order on the XCDs (logical_block).
template <class F, int BYI>
__global__ __launch_bounds__(64 * (BYI + 3)) void batch_pass_kernel(const BatchLat *__restrict__ lats,
                                                                    const BatchBox *__restrict__ boxes,
                                                                    const int *__restrict__ nboxes, int s, int parity,
                                                                    int zc, int remap) {
  using S = typename F::S;
  using T = typename Codec<S>::T;
  __shared__ S ring[kRingPlanes * Sweep2Tile<F, BYI>::kPlane];
  const int nb = *nboxes;
  if (int(blockIdx.x) >= nb) return;  // uniform over the workgroup
  const BatchBox bx = boxes[logical_block(blockIdx.x, unsigned(nb), remap, 1u)];
  const BatchLat &L = lats[bx.lat];
  Sweep2Args<T> a;
  a.nx = int(L.nx);
  a.ny = int(L.ny);
  a.nz = int(L.nz);
  a.pop_stride = L.pop_stride;
  a.row_stride = L.row_stride;
  a.tiles_x = 0;  // the box is given
  a.tiles_y = 0;
  a.zc = zc;
  a.xcd_remap = 0;
  a.key0 = step_key(L.step_base + unsigned(s));
  a.key1 = step_key(L.step_base + unsigned(s) + 1u);
  a.p = lattice_params<T>(L);
  // global (not flat) accesses: the addresses come from memory
  const global_ptr<const S> src = (global_ptr<const S>)(L.buf[parity]);
  const global_ptr<S> dst = (global_ptr<S>)(L.buf[parity ^ 1]);
  sweep2_box<F, BYI, global_ptr<const S>, global_ptr<S>>(src, dst, a, bx.tx, bx.ty, bx.tz, ring);
}

// own: the grid is the tile table's capacity, one workgroup per entry.
template <class F, int BX>
static void launch_batch_sweep_t(const BatchLat *lats, const BatchTile *tiles, const int *nt, int s, int parity,
                                 float *partials, int grid, bool own, hipStream_t st) {
  if (partials)  // the measure: one workgroup per tile
    batch_sweep_kernel<F, BX, true, true><<<dim3(grid), dim3(BX), 0, st>>>(lats, tiles, nt, s, parity, partials);
  else if (own)
    batch_sweep_kernel<F, BX, false, true><<<dim3(grid), dim3(BX), 0, st>>>(lats, tiles, nt, s, parity, nullptr);
  else
    batch_sweep_kernel<F, BX, false, false><<<dim3(grid), dim3(BX), 0, st>>>(lats, tiles, nt, s, parity, nullptr);
}

// partials: non-null for the step that ends a chunk, with one workgroup per
// tile (the per-wave maxima of the convergence measure, bx / 64 per tile).
static hipError_t launch_batch_sweep(int storage, int bx, const BatchLat *lats, const BatchTile *tiles, const int *nt,
                                     int s, int parity, float *partials, int grid, bool own, hipStream_t st) {
#define LBM_CASE(ST, F, B)                                                                 \
  case ST * 1000 + B:                                                                      \
    launch_batch_sweep_t<F, B>(lats, tiles, nt, s, parity, partials, grid, own, st);       \
    break;
  switch (storage * 1000 + bx) {
    LBM_CASE(kStoreF64, FormF64, 128)
    LBM_CASE(kStoreF64, FormF64, 256)
    LBM_CASE(kStoreF32, FormF32, 128)
    LBM_CASE(kStoreF32, FormF32, 256)
    LBM_CASE(kStoreF16, FormF16, 128)
    LBM_CASE(kStoreF16, FormF16, 256)
    LBM_CASE(kStoreF16SR, FormF16SR, 128)
    LBM_CASE(kStoreF16SR, FormF16SR, 256)
    default: return hipErrorInvalidValue;
  }
#undef LBM_CASE
  return hipGetLastError();
}

// Interior rows of the two-step pass's tiles for a storage form.
static int pass_rows(int storage) {
  switch (storage) {
    case kStoreF64: return Sweep2Rows<FormF64>::kBYI;
    case kStoreF32: return Sweep2Rows<FormF32>::kBYI;
    case kStoreF16: return Sweep2Rows<FormF16>::kBYI;
    default: return Sweep2Rows<FormF16SR>::kBYI;
  }
}

template <class F>
static void launch_batch_pass_t(const BatchLat *lats, const BatchBox *boxes, const int *nb, int s, int parity, int zc,
                                int remap, int grid, hipStream_t st) {
  constexpr int BYI = Sweep2Rows<F>::kBYI;
  batch_pass_kernel<F, BYI><<<dim3(grid), dim3(Sweep2Tile<F, BYI>::kThreads), 0, st>>>(lats, boxes, nb, s, parity,
                                                                                     zc, remap);
}

static hipError_t launch_batch_pass(int storage, const BatchLat *lats, const BatchBox *boxes, const int *nb, int s,
                                    int parity, int zc, int remap, int grid, hipStream_t st) {
  switch (storage) {
    case kStoreF64: launch_batch_pass_t<FormF64>(lats, boxes, nb, s, parity, zc, remap, grid, st); break;
    case kStoreF32: launch_batch_pass_t<FormF32>(lats, boxes, nb, s, parity, zc, remap, grid, st); break;
    case kStoreF16: launch_batch_pass_t<FormF16>(lats, boxes, nb, s, parity, zc, remap, grid, st); break;
    case kStoreF16SR: launch_batch_pass_t<FormF16SR>(lats, boxes, nb, s, parity, zc, remap, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_batch_delta(int storage, const BatchLat *lats, const BatchTile *tiles, const int *nt,
                                     unsigned *delta, int grid, hipStream_t s) {
  switch (storage) {
    case kStoreF64: batch_delta_kernel<double><<<dim3(grid), dim3(256), 0, s>>>(lats, tiles, nt, delta); break;
    case kStoreF32: batch_delta_kernel<float><<<dim3(grid), dim3(256), 0, s>>>(lats, tiles, nt, delta); break;
    case kStoreF16:
    case kStoreF16SR: batch_delta_kernel<_Float16><<<dim3(grid), dim3(256), 0, s>>>(lats, tiles, nt, delta); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbm

// ---------------------------------------------------------------------------
// Host runtime.
// ---------------------------------------------------------------------------
namespace {

#define bfail lbm::set_error

#define LBM_BHIP(call, what)                                                                 \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return bfail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kNumStorage = 4;
constexpr int kMinTileNodes = 256;
constexpr int kMaxLanes = 8;
constexpr size_t kResultCacheBytes = size_t(4) << 30;  // page-locked result blocks kept for reuse

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Layout of a job's populations.  Row-major (the 19 populations of each
// x-row together) where a row is a whole number of 128-byte lines: the sweep
// then streams through a few nearby regions per tile instead of 38 regions
// one population apart.  Otherwise population-major: there the flat node
// walk of the batch sweep keeps every wave on whole lines, while row-major
// rows would end inside lines (written in parts) or, padded, leave lanes
// idle -- on 64 ducts of nx 32..256 the batch sweep ran at 17.4 GLUPS
// row-major unpadded, 27.2 padded with row-aligned slots, 32.4 this way.
int batch_layout_kind(int nx, size_t esize) {
  return (size_t(nx) * esize) % 128 == 0 ? LBM_LAYOUT_ROW_MAJOR : LBM_LAYOUT_POPULATION_MAJOR;
}
lbm::PopLayout layout_of(int kind, size_t nodes, int nx, size_t esize) {
  return kind == LBM_LAYOUT_ROW_MAJOR ? lbm::row_major(nx, esize) : lbm::population_major(nodes, nx);
}

// First-fit allocator over one device allocation; free blocks are kept
// sorted by offset and coalesced.
class Pool {
 public:
  void reset(size_t cap) {
    cap_ = cap;
    free_.clear();
    free_[0] = cap;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t capacity() const { return cap_; }

 private:
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

size_t job_bytes(const lbm_job &j, int layout) {
  const size_t N = size_t(j.nx) * j.ny * j.nz;
  const size_t esize = lbm_element_bytes(j.storage);
  return 2 * align_up(lbm::buffer_elements(layout, j.nx, j.ny, j.nz, esize) * esize) +
         align_up(3 * N * sizeof(float));
}

// Host memory block, page-locked when the runtime grants it (a
// device-to-host copy into fresh pageable memory runs at about 4 GB/s on this
// host, page faults included, into page-locked memory at about 40 GB/s),
// pageable otherwise.
class HostBlock {
 public:
  HostBlock() = default;
  HostBlock(const HostBlock &) = delete;
  HostBlock &operator=(const HostBlock &) = delete;
  HostBlock(HostBlock &&o) noexcept : p_(o.p_), bytes_(o.bytes_), pinned_(o.pinned_) { o.p_ = nullptr, o.bytes_ = 0; }
  HostBlock &operator=(HostBlock &&o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_, bytes_ = o.bytes_, pinned_ = o.pinned_;
      o.p_ = nullptr, o.bytes_ = 0;
    }
    return *this;
  }
  ~HostBlock() { release(); }
  bool allocate(size_t bytes, bool need_pinned = false) {
    release();
    void *p = nullptr;
    pinned_ = hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess;
    if (!pinned_) {
      (void)hipGetLastError();
      if (need_pinned) return false;
      p = ::operator new(bytes, std::nothrow);
      if (!p) return false;
    }
    p_ = p;
    bytes_ = bytes;
    return true;
  }
  void release() {
    if (p_) {
      if (pinned_)
        (void)hipHostFree(p_);
      else
        ::operator delete(p_);
    }
    p_ = nullptr;
    bytes_ = 0;
  }
  template <class T>
  T *as() const {
    return static_cast<T *>(p_);
  }
  size_t bytes() const { return bytes_; }

 private:
  void *p_ = nullptr;
  size_t bytes_ = 0;
  bool pinned_ = false;
};

struct Job {
  lbm_job spec;
  size_t nodes = 0;
  int state = LBM_JOB_QUEUED;
  int slot = -1;
  int lane = -1;  // lane whose chunk in flight steps this job, or -1
  size_t off = 0, bytes = 0;
  int steps = 0;
  double delta = INFINITY;
  int converged = 0;
  int waited = 0;   // chunks spent at the head of the queue without fitting
  int skipped = 0;  // consecutive scheduling rounds resident, idle and not stepped
  int layout = LBM_LAYOUT_POPULATION_MAJOR;  // chosen at submission
  lbm::SweepConfig cfg{};                    // single-lattice sweep of the job (set at admission)
  HostBlock result;  // moments at retirement: rho [N], then u [3][N], in double
};

struct Shape {
  int block_x = 256, tile_nodes = 256, grid = 0;  // grid 0: one workgroup per tile
};

// A tuned configuration: the single step's shape, and the two-step pass's z
// planes and box order.
struct Tuned {
  Shape shape;
  int zc = 32, remap = 1;
};

// Autotune results shared by every batch in the process, keyed by a coarse
// description of the resident work (storage mix, log2 of the node count,
// steps per pass); batches on different threads share it under a lock.
std::map<long long, Tuned> g_tuned;
std::mutex g_tuned_mutex;

// One lane: a stream with its own descriptor and tile tables, so that the
// chunks of different lanes run on the device at the same time.  Host-side
// staging of the tables and of the convergence maxima is page-locked; it is
// written only while the lane is idle (its previous chunk, including these
// copies, has completed).
struct Lane {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<int> slots;  // slots the chunk in flight steps
  lbm::BatchLat *d_lats = nullptr;
  unsigned *d_delta = nullptr;
  int *d_ntiles = nullptr;  // tile counts per storage form, then box counts
  lbm::BatchTile *d_tiles[kNumStorage] = {nullptr, nullptr, nullptr, nullptr};
  size_t tile_cap[kNumStorage] = {0, 0, 0, 0};
  lbm::BatchBox *d_boxes[kNumStorage] = {nullptr, nullptr, nullptr, nullptr};  // the two-step pass's boxes
  size_t box_cap[kNumStorage] = {0, 0, 0, 0};
  HostBlock h_lats, h_delta, h_ntiles, h_tiles[kNumStorage], h_boxes[kNumStorage];
  int ntiles[kNumStorage] = {0, 0, 0, 0};
  int nboxes[kNumStorage] = {0, 0, 0, 0};
  // per-wave maxima of the convergence measure taken by a chunk's last step:
  // for a graph chunk 4 per tile-table entry of each storage form (form s
  // from part_off[s]), for a chunk of one job its single sweep's
  float *d_part = nullptr;
  size_t part_cap = 0, part_off[kNumStorage] = {0, 0, 0, 0};
  // Jobs (slot, job id) the tile tables describe: a slot reused by a later
  // job has other extents, so the tables follow the job ids, not the slots.
  std::vector<std::pair<int, int>> table_jobs;
  int table_tile_nodes = 0, table_pass = 0, table_zc = 0;
  // captured chunks by (storage forms present, chunk steps, block_x, grid,
  // steps per pass, z planes, box order)
  std::map<std::tuple<unsigned, int, int, int, int, int, int>, hipGraphExec_t> graphs;
};

}  // namespace

struct lbm_batch {
  hipStream_t user_stream = nullptr;
  int num_cu = 256;
  char *pool_base = nullptr;
  Pool pool;
  int chunk_steps = 100;
  int max_jobs = 0;
  Shape shape;
  // Steps per pass: 1, one step per launch; 2, two steps per pass over the
  // jobs of every chunk (every job row-major), z ranges of pass_zc planes per
  // workgroup, box order pass_remap on the XCDs.
  int pass_steps = 1, pass_zc = 32, pass_remap = 1;
  std::map<int, Job> jobs;
  std::deque<int> queue;
  std::vector<int> slot_job;           // slot -> job id (-1 free)
  std::vector<lbm::BatchLat> lat;      // slot -> descriptor (step_base set at upload)
  int next_id = 1;
  int policy = LBM_BATCH_LOCKSTEP;  // which resident jobs a chunk steps
  size_t fill_nodes = 0;            // LBM_BATCH_SHORTEST_FIRST: nodes a chunk steps at least
  std::vector<Lane> lanes;
  std::vector<HostBlock> result_cache;  // released result blocks, reused by later retirements
  size_t result_cache_bytes = 0;
  lbm_batch_stats stats{};
  // Admitted jobs are initialised on a stream of their own, so that a new
  // job does not wait behind a chunk in flight; every chunk waits for the
  // initialisations enqueued before it.
  hipStream_t init_stream = nullptr;
  hipEvent_t init_done = nullptr;
  bool init_recorded = false;
};

namespace {

void drop_graphs(Lane &ln) {
  for (auto &kv : ln.graphs) (void)hipGraphExecDestroy(kv.second);
  ln.graphs.clear();
}

void free_lane(Lane &ln) {
  if (ln.stream) (void)hipStreamSynchronize(ln.stream);
  drop_graphs(ln);
  if (ln.d_lats) (void)hipFree(ln.d_lats);
  if (ln.d_delta) (void)hipFree(ln.d_delta);
  if (ln.d_ntiles) (void)hipFree(ln.d_ntiles);
  for (int s = 0; s < kNumStorage; ++s) {
    if (ln.d_tiles[s]) (void)hipFree(ln.d_tiles[s]);
    if (ln.d_boxes[s]) (void)hipFree(ln.d_boxes[s]);
  }
  if (ln.d_part) (void)hipFree(ln.d_part);
  if (ln.done) (void)hipEventDestroy(ln.done);
  if (ln.own_stream && ln.stream) (void)hipStreamDestroy(ln.stream);
  ln = Lane();
}

lbm_status init_lane(lbm_batch *B, Lane &ln, hipStream_t given) {
  if (given) {
    ln.stream = given;
  } else {
    // Graph capture needs a stream other than the null stream; every stream
    // keeps the default priority.
    LBM_BHIP(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking), "stream creation");
    ln.own_stream = true;
  }
  LBM_BHIP(hipEventCreateWithFlags(&ln.done, hipEventDisableTiming), "event creation");
  const size_t mj = size_t(B->max_jobs);
  bool ok = hipMalloc(&ln.d_lats, sizeof(lbm::BatchLat) * mj) == hipSuccess &&
            hipMalloc(&ln.d_delta, sizeof(unsigned) * mj) == hipSuccess &&
            hipMalloc(&ln.d_ntiles, sizeof(int) * 2 * kNumStorage) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return bfail(LBM_ERR_OOM, "device tables of a lane could not be allocated");
  }
  if (!ln.h_lats.allocate(sizeof(lbm::BatchLat) * mj, true) || !ln.h_delta.allocate(sizeof(unsigned) * mj, true) ||
      !ln.h_ntiles.allocate(sizeof(int) * 2 * kNumStorage, true))
    return bfail(LBM_ERR_OOM, "page-locked staging of a lane could not be allocated");
  std::memset(ln.h_lats.as<void>(), 0, ln.h_lats.bytes());
  return LBM_OK;
}

// Room for n entries in one of a lane's device tables (tiles or boxes of a
// storage form) and its page-locked staging.  A new device table invalidates
// the lane's captured graphs (their launches hold the old address and take
// the old capacity as their grid).  Only called while the lane is idle.
template <class E>
lbm_status ensure_table(Lane &ln, E *&d, size_t &cap, HostBlock &h, size_t n, const char *what) {
  if (n <= cap) return LBM_OK;
  size_t c = std::max<size_t>(n, 2 * cap);
  c = std::max<size_t>(c, 1024);
  drop_graphs(ln);
  if (d) (void)hipFree(d);
  d = nullptr;
  cap = 0;
  if (hipMalloc(&d, sizeof(E) * c) != hipSuccess) {
    (void)hipGetLastError();
    d = nullptr;
    return bfail(LBM_ERR_OOM, "%s table of %zu entries could not be allocated", what, c);
  }
  if (!h.allocate(sizeof(E) * c, true))
    return bfail(LBM_ERR_OOM, "page-locked %s staging of %zu entries could not be allocated", what, c);
  cap = c;
  return LBM_OK;
}

// Room for n per-wave maxima in a lane's partials (reallocation drops the
// lane's graphs).  Only called while the lane is idle.
lbm_status ensure_partials(Lane &ln, size_t n) {
  if (n <= ln.part_cap) return LBM_OK;
  const size_t c = std::max<size_t>(n, 2 * ln.part_cap);
  drop_graphs(ln);
  if (ln.d_part) (void)hipFree(ln.d_part);
  ln.d_part = nullptr;
  ln.part_cap = 0;
  if (hipMalloc(&ln.d_part, sizeof(float) * c) != hipSuccess) {
    (void)hipGetLastError();
    ln.d_part = nullptr;
    return bfail(LBM_ERR_OOM, "partials of %zu entries could not be allocated", c);
  }
  ln.part_cap = c;
  return LBM_OK;
}

unsigned present_mask(const Lane &ln) {
  unsigned m = 0;
  for (int s = 0; s < kNumStorage; ++s)
    if (ln.ntiles[s] > 0) m |= 1u << s;
  return m;
}

// Tables of a lane for the jobs in `slots`: the descriptors (with the step
// counts as step_base) always, the tile lists when the job set or the tile
// size changed.  Asynchronous copies from page-locked staging on the lane's
// stream; the lane is idle.
lbm_status upload_tables(lbm_batch *B, Lane &ln, const std::vector<int> &slots) {
  std::vector<std::pair<int, int>> jobs;
  for (int slot : slots) jobs.push_back({slot, B->slot_job[slot]});
  const bool pass2 = B->pass_steps == 2;
  if (jobs != ln.table_jobs || ln.table_tile_nodes != B->shape.tile_nodes || ln.table_pass != B->pass_steps ||
      ln.table_zc != B->pass_zc) {
    std::vector<lbm::BatchTile> tiles[kNumStorage];
    std::vector<lbm::BatchBox> boxes[kNumStorage];
    const unsigned tn = unsigned(B->shape.tile_nodes);
    for (int slot : slots) {
      const Job &J = B->jobs.at(B->slot_job[slot]);
      const int st = J.spec.storage;
      const unsigned S = unsigned(size_t(B->lat[slot].slot_row) * J.spec.ny * J.spec.nz);  // slots of the job
      for (unsigned n0 = 0; n0 < S; n0 += tn) tiles[st].push_back({slot, n0, std::min(S, n0 + tn)});
      if (!pass2) continue;
      if (J.layout != LBM_LAYOUT_ROW_MAJOR)
        return bfail(LBM_ERR_STATE, "job %d is not row-major: two steps per pass need every job row-major",
                     B->slot_job[slot]);
      // boxes z range by z range, row of tiles by row of tiles
      const unsigned by = unsigned(lbm::pass_rows(st)), zc = unsigned(B->pass_zc);
      const unsigned tx = (unsigned(J.spec.nx) + 63u) / 64u, ty = (unsigned(J.spec.ny) + by - 1u) / by;
      const unsigned tz = (unsigned(J.spec.nz) + zc - 1u) / zc;
      for (unsigned z = 0; z < tz; ++z)
        for (unsigned y = 0; y < ty; ++y)
          for (unsigned x = 0; x < tx; ++x) boxes[st].push_back({slot, x, y, z});
    }
    int *counts = ln.h_ntiles.as<int>();
    for (int s = 0; s < kNumStorage; ++s) {
      lbm_status st = ensure_table(ln, ln.d_tiles[s], ln.tile_cap[s], ln.h_tiles[s], tiles[s].size(), "tile");
      if (st == LBM_OK) st = ensure_table(ln, ln.d_boxes[s], ln.box_cap[s], ln.h_boxes[s], boxes[s].size(), "box");
      if (st != LBM_OK) return st;
      ln.ntiles[s] = int(tiles[s].size());
      ln.nboxes[s] = int(boxes[s].size());
      if (!tiles[s].empty()) {
        std::memcpy(ln.h_tiles[s].as<void>(), tiles[s].data(), tiles[s].size() * sizeof(lbm::BatchTile));
        LBM_BHIP(hipMemcpyAsync(ln.d_tiles[s], ln.h_tiles[s].as<void>(), tiles[s].size() * sizeof(lbm::BatchTile),
                                hipMemcpyHostToDevice, ln.stream),
                 "upload tiles");
      }
      if (!boxes[s].empty()) {
        std::memcpy(ln.h_boxes[s].as<void>(), boxes[s].data(), boxes[s].size() * sizeof(lbm::BatchBox));
        LBM_BHIP(hipMemcpyAsync(ln.d_boxes[s], ln.h_boxes[s].as<void>(), boxes[s].size() * sizeof(lbm::BatchBox),
                                hipMemcpyHostToDevice, ln.stream),
                 "upload boxes");
      }
      counts[s] = ln.ntiles[s];
      counts[kNumStorage + s] = ln.nboxes[s];
    }
    LBM_BHIP(hipMemcpyAsync(ln.d_ntiles, counts, sizeof(int) * 2 * kNumStorage, hipMemcpyHostToDevice, ln.stream),
             "upload tile and box counts");
    size_t np = 0;
    for (int s = 0; s < kNumStorage; ++s) {
      ln.part_off[s] = np;
      np += 4 * ln.tile_cap[s];
    }
    lbm_status st = ensure_partials(ln, np);
    if (st != LBM_OK) return st;
    ln.table_jobs = jobs;
    ln.table_tile_nodes = B->shape.tile_nodes;
    ln.table_pass = B->pass_steps;
    ln.table_zc = B->pass_zc;
  }
  lbm::BatchLat *h = ln.h_lats.as<lbm::BatchLat>();
  int lo = B->max_jobs, hi = -1;
  for (int slot : slots) {
    h[slot] = B->lat[slot];
    h[slot].step_base = unsigned(B->jobs.at(B->slot_job[slot]).steps);
    lo = std::min(lo, slot);
    hi = std::max(hi, slot);
  }
  if (hi >= lo)
    LBM_BHIP(hipMemcpyAsync(ln.d_lats + lo, h + lo, sizeof(lbm::BatchLat) * size_t(hi - lo + 1),
                            hipMemcpyHostToDevice, ln.stream),
             "upload lattices");
  return LBM_OK;
}

// Passes of two steps in a sequence of nsteps (even) steps that starts and
// ends with the state in buf[0]: each pass leaves the state in the other
// buffer, each single step too, so the count of passes has the parity of
// nsteps / 2 ... minus one when that is odd, and two single steps close the
// sequence (10 steps: 4 passes and 2 single steps; 100 steps: 50 passes).
int passes_in(int nsteps) {
  const int m = nsteps / 2;
  return m % 2 == 0 ? m : m - 1;
}

// Enqueue nsteps (even) steps with indices first..first+nsteps-1 of a
// sequence that starts at each lattice's step_base, the state in buf[0]
// before and after.  With two steps per pass: passes_in(nsteps) passes over
// the lane's boxes, then single steps; else single steps.  Grid of a single
// step: the shape's persistent workgroups, or (grid 0) one workgroup per
// entry of the lane's tile table -- its capacity, which only changes when
// the table is reallocated, and then the lane's graphs are dropped;
// workgroups past the current tile count exit at once.  A pass launches one
// workgroup per entry of the box table in the same way.  measure: the
// sequence ends a chunk and its last step (a single step with one workgroup
// per tile) also takes the convergence measure into the lane's partials.
lbm_status launch_steps(lbm_batch *B, Lane &ln, int nsteps, int first, bool measure) {
  const int P = B->pass_steps == 2 ? passes_in(nsteps) : 0;
  for (int i = 0; i < P; ++i)
    for (int s = 0; s < kNumStorage; ++s)
      if (ln.nboxes[s] > 0)
        LBM_BHIP(lbm::launch_batch_pass(s, ln.d_lats, ln.d_boxes[s], ln.d_ntiles + kNumStorage + s, first + 2 * i,
                                        i & 1, B->pass_zc, B->pass_remap, int(ln.box_cap[s]), ln.stream),
                 "batch pass launch");
  for (int j = 2 * P; j < nsteps; ++j) {
    const int parity = (j - P) & 1;  // buffer flips so far: P passes and j - 2P single steps
    for (int s = 0; s < kNumStorage; ++s)
      if (ln.ntiles[s] > 0) {
        const int grid = B->shape.grid > 0 ? B->shape.grid : int(ln.tile_cap[s]);
        LBM_BHIP(lbm::launch_batch_sweep(s, B->shape.block_x, ln.d_lats, ln.d_tiles[s], ln.d_ntiles + s, first + j,
                                         parity, measure && j == nsteps - 1 ? ln.d_part + ln.part_off[s] : nullptr,
                                         grid, B->shape.grid == 0, ln.stream),
                 "batch sweep launch");
      }
  }
  return LBM_OK;
}

// Whether a chunk's last step takes the convergence measure: it is a single
// step (not a pass of two), of one job alone or with one workgroup per tile.
bool measured_in_last_step(const lbm_batch *B, bool solo) {
  return (B->pass_steps != 2 || B->chunk_steps > 2 * passes_in(B->chunk_steps)) && (solo || B->shape.grid == 0);
}

// A chunk that steps a single job: plain launches of the single-lattice
// sweep on the job's buffers (row-aligned blocks; bitwise the batch sweep's
// results), one per step, each with the job's own step index; the last one
// also takes the convergence measure.
lbm_status run_solo_chunk(lbm_batch *B, Lane &ln, int slot) {
  const Job &J = B->jobs.at(B->slot_job[slot]);
  const lbm::BatchLat &L = B->lat[slot];
  lbm::SweepConfig c = J.cfg;
  // with two steps per pass, passes of the single-lattice two-step kernel
  // first (the same order of buffers as launch_steps; the job is row-major)
  const int P = B->pass_steps == 2 ? passes_in(B->chunk_steps) : 0;
  for (int i = 0; i < P; ++i) {
    c.step = unsigned(J.steps + 2 * i);
    LBM_BHIP(lbm::launch_sweep2(c, B->pass_zc, 0, L.buf[i & 1], L.buf[(i & 1) ^ 1], ln.stream), "pass launch");
  }
  for (int s = 2 * P; s < B->chunk_steps; ++s) {
    const int q = (s - P) & 1;
    c.step = unsigned(J.steps + s);
    if (s == B->chunk_steps - 1 && measured_in_last_step(B, true)) {
      lbm_status st = ensure_partials(ln, lbm::sweep_delta_partials(c));
      if (st != LBM_OK) return st;
      LBM_BHIP(lbm::launch_sweep_delta(c, L.buf[q], L.buf[q ^ 1], L.snap, L.inv_uref, ln.d_part, ln.d_delta + slot,
                                       ln.stream),
               "sweep launch");
    }
    else
      LBM_BHIP(lbm::launch_sweep(c, L.buf[q], L.buf[q ^ 1], false, ln.stream), "sweep launch");
  }
  return LBM_OK;
}

lbm_status run_graph_chunk(lbm_batch *B, Lane &ln) {
  const unsigned mask = present_mask(ln);
  if (!mask) return LBM_OK;
  const auto key = std::make_tuple(mask, B->chunk_steps, B->shape.block_x, B->shape.grid, B->pass_steps, B->pass_zc,
                                   B->pass_remap);
  auto it = ln.graphs.find(key);
  if (it == ln.graphs.end()) {
    hipGraph_t graph;
    LBM_BHIP(hipStreamBeginCapture(ln.stream, hipStreamCaptureModeThreadLocal), "begin capture");
    lbm_status st = launch_steps(B, ln, B->chunk_steps, 0, measured_in_last_step(B, false));
    hipError_t e = hipStreamEndCapture(ln.stream, &graph);
    if (st != LBM_OK) return st;
    if (e != hipSuccess) return bfail(LBM_ERR_HIP, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return bfail(LBM_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    it = ln.graphs.emplace(key, exec).first;
  }
  LBM_BHIP(hipGraphLaunch(it->second, ln.stream), "graph launch");
  return LBM_OK;
}

// Host block for a retiring job's moments: a cached block large enough, else
// a new one.
bool take_result_block(lbm_batch *B, HostBlock &out, size_t bytes) {
  int best = -1;
  for (int i = 0; i < int(B->result_cache.size()); ++i)
    if (B->result_cache[i].bytes() >= bytes &&
        (best < 0 || B->result_cache[i].bytes() < B->result_cache[best].bytes()))
      best = i;
  if (best >= 0) {
    B->result_cache_bytes -= B->result_cache[best].bytes();
    out = std::move(B->result_cache[best]);
    B->result_cache.erase(B->result_cache.begin() + best);
    return true;
  }
  return out.allocate(bytes);
}

void give_back_result_block(lbm_batch *B, HostBlock &&blk) {
  if (!blk.bytes()) return;
  if (B->result_cache_bytes + blk.bytes() > kResultCacheBytes) return;  // freed with blk
  B->result_cache_bytes += blk.bytes();
  B->result_cache.push_back(std::move(blk));
}

// Moments of a finished job into host memory, then release its device
// memory.  The moments are written in double (rho [N], then u [3][N]) into
// the job's idle population buffer (it holds at least 38 N bytes), then
// copied to the host.  Synchronizes the lane's stream.
lbm_status retire(lbm_batch *B, int id, Lane &ln) {
  Job &J = B->jobs.at(id);
  const size_t N = J.nodes;
  if (!take_result_block(B, J.result, 4 * N * sizeof(double)))
    return bfail(LBM_ERR_OOM, "host memory for the moments of job %d", id);
  const lbm::BatchLat &L = B->lat[J.slot];
  double *scratch = static_cast<double *>(L.buf[1]);
  LBM_BHIP(lbm::launch_moments(J.spec.storage, L.buf[0],
                               layout_of(J.layout, N, J.spec.nx, lbm_element_bytes(J.spec.storage)), 0, N, scratch,
                               scratch + N, nullptr, 1024, ln.stream),
           "moments");
  LBM_BHIP(hipMemcpyAsync(J.result.as<void>(), scratch, 4 * N * sizeof(double), hipMemcpyDeviceToHost, ln.stream),
           "copy moments");
  LBM_BHIP(hipStreamSynchronize(ln.stream), "moments");
  B->pool.release(J.off, J.bytes);
  B->slot_job[J.slot] = -1;
  std::memset(&B->lat[J.slot], 0, sizeof(lbm::BatchLat));
  J.slot = -1;
  J.state = LBM_JOB_DONE;
  return LBM_OK;
}

// Admit queued jobs in arrival order while memory and slots allow.  A job may
// pass the head of the queue only while the head has waited fewer than four
// chunks, so large jobs are not starved by a stream of small ones.
lbm_status admit(lbm_batch *B) {
  bool head_blocked = false;
  for (auto it = B->queue.begin(); it != B->queue.end();) {
    Job &J = B->jobs.at(*it);
    int slot = -1;
    for (int s = 0; s < B->max_jobs; ++s)
      if (B->slot_job[s] < 0) {
        slot = s;
        break;
      }
    size_t off = 0;
    if (slot < 0 || !B->pool.alloc(J.bytes, &off)) {
      if (it == B->queue.begin()) {
        ++J.waited;
        head_blocked = J.waited >= 4;
      }
      if (head_blocked || slot < 0) break;
      ++it;
      continue;
    }
    const size_t N = J.nodes;
    const size_t esize = lbm_element_bytes(J.spec.storage);
    const size_t elems = lbm::buffer_elements(J.layout, J.spec.nx, J.spec.ny, J.spec.nz, esize);
    const size_t buf_bytes = align_up(elems * esize);
    lbm::BatchLat L;
    std::memset(&L, 0, sizeof(L));
    L.buf[0] = B->pool_base + off;
    L.buf[1] = B->pool_base + off + buf_bytes;
    L.snap = reinterpret_cast<float *>(B->pool_base + off + 2 * buf_bytes);
    L.nx = unsigned(J.spec.nx);
    L.ny = unsigned(J.spec.ny);
    L.nz = unsigned(J.spec.nz);
    L.N = unsigned(N);
    L.buf_elems = unsigned(elems);
    const lbm::PopLayout lay = layout_of(J.layout, N, J.spec.nx, esize);
    L.pop_stride = unsigned(lay.pop_stride);
    L.row_stride = unsigned(lay.row_stride);
    L.slot_row = J.layout == LBM_LAYOUT_ROW_MAJOR ? unsigned(lay.pop_stride)  // the padded row pitch
                                                  : unsigned(J.spec.nx);
    L.bc_mask = J.spec.bc_mask;
    L.p_mask = J.spec.pressure_mask;
    L.omega = 1.0 / J.spec.tau;
    std::memcpy(L.v, J.spec.bc_velocity, sizeof(L.v));
    for (int f = 0; f < 6; ++f) {
      if (!((L.p_mask >> f) & 1u)) continue;
      // pressure face: keep the tangential velocity only
      const double un = L.v[f][0] * lbm::kFaceNormal[f][0] + L.v[f][1] * lbm::kFaceNormal[f][1] + L.v[f][2] * lbm::kFaceNormal[f][2];
      for (int d = 0; d < 3; ++d) L.v[f][d] -= un * lbm::kFaceNormal[f][d];
      L.rho_p[f] = J.spec.bc_rho[f];
    }
    for (int d = 0; d < 3; ++d) L.tau_f[d] = J.spec.tau * J.spec.force[d];
    L.inv_uref = 1.0 / J.spec.u_ref;
    // the same lattice as a single-lattice sweep (a chunk that steps this job alone)
    lbm::SweepConfig &c = J.cfg;
    c = lbm::SweepConfig{};
    c.storage = J.spec.storage;
    c.nx = J.spec.nx;
    c.ny = J.spec.ny;
    c.nz = J.spec.nz;
    c.layout = lay;
    c.tau = J.spec.tau;
    c.bc_mask = L.bc_mask;
    c.p_mask = L.p_mask;
    std::memcpy(c.v, L.v, sizeof(c.v));
    std::memcpy(c.rho_p, L.rho_p, sizeof(c.rho_p));
    for (int d = 0; d < 3; ++d) c.force[d] = J.spec.force[d];
    c.block_x = lbm::default_block_x(J.spec.nx);
    c.nodes_per_thread = 1;
    c.xcd_remap = LBM_XCD_SLABS;
    B->lat[slot] = L;
    B->slot_job[slot] = *it;
    const double zero[3] = {0.0, 0.0, 0.0};
    LBM_BHIP(lbm::launch_init(J.spec.storage, L.buf[0], N, lay, J.spec.rho0, zero, B->init_stream), "init launch");
    const size_t n3 = 3 * N;
    lbm::fill_float_kernel<<<dim3(unsigned((n3 + 255) / 256)), dim3(256), 0, B->init_stream>>>(L.snap, n3, 0.0f);
    LBM_BHIP(hipGetLastError(), "snapshot fill");
    LBM_BHIP(hipEventRecord(B->init_done, B->init_stream), "event");
    B->init_recorded = true;
    J.off = off;
    J.slot = slot;
    J.state = LBM_JOB_RUNNING;
    it = B->queue.erase(it);
  }
  return LBM_OK;
}

double job_nodes(const Job &J) { return double(J.nodes); }

// Resident jobs not in flight, grouped for the idle lanes.
//   Lockstep: all of them; with several idle lanes, each job (largest first)
//   goes to the lane with the fewest nodes so far.
//   Shortest first: jobs left out for kMaxSkipped rounds, then the others in
//   order of remaining work (nodes x steps left to max_steps, ties by slot).
//   Each idle lane takes the next job; a job below fill_nodes nodes takes
//   further jobs below fill_nodes with it until the lane holds fill_nodes
//   nodes.  The rest wait, resident.  Small jobs then step at their own pace
//   instead of a large co-resident job's, and a large job waits, but not for
//   ever.
//   Large in order: jobs of at least fill_nodes nodes are large.  While no
//   large job is in flight, the earliest submitted large job takes an idle
//   lane (large jobs run one at a time, in arrival order, so a later one
//   never slows an earlier one down); the other idle lanes take small jobs,
//   one each, in order of remaining work (left-out ones first, as above).
constexpr int kMaxSkipped = 50;
std::vector<std::pair<int, std::vector<int>>> plan_chunks(lbm_batch *B) {
  std::vector<int> idle;
  for (int l = 0; l < int(B->lanes.size()); ++l)
    if (!B->lanes[l].busy) idle.push_back(l);
  std::vector<int> cand;
  for (int slot = 0; slot < B->max_jobs; ++slot) {
    const int id = B->slot_job[slot];
    if (id >= 0 && B->jobs.at(id).lane < 0) cand.push_back(slot);
  }
  std::vector<std::pair<int, std::vector<int>>> plan;
  if (idle.empty() || cand.empty()) return plan;
  for (int l : idle) plan.push_back({l, {}});
  auto job_at = [&](int slot) -> Job & { return B->jobs.at(B->slot_job[slot]); };
  if (B->policy == LBM_BATCH_LOCKSTEP) {
    std::vector<int> order = cand;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return job_nodes(job_at(a)) > job_nodes(job_at(b)); });
    std::vector<double> load(plan.size(), 0.0);
    for (int slot : order) {
      const size_t g = size_t(std::min_element(load.begin(), load.end()) - load.begin());
      plan[g].second.push_back(slot);
      load[g] += job_nodes(job_at(slot));
    }
  } else if (B->policy == LBM_BATCH_LARGE_IN_ORDER) {
    const double big = double(B->fill_nodes);
    bool large_running = false;
    for (int slot = 0; slot < B->max_jobs; ++slot) {
      const int id = B->slot_job[slot];
      if (id >= 0 && B->jobs.at(id).lane >= 0 && job_nodes(B->jobs.at(id)) >= big) large_running = true;
    }
    int first_large = -1;  // earliest submitted (smallest id) large candidate
    std::vector<std::pair<std::pair<int, double>, int>> small;  // ((not forced, work), slot)
    for (int slot : cand) {
      const Job &J = job_at(slot);
      if (job_nodes(J) >= big) {
        if (first_large < 0 || B->slot_job[slot] < B->slot_job[first_large]) first_large = slot;
      } else {
        const double work = job_nodes(J) * double(std::max(0, J.spec.max_steps - J.steps));
        small.push_back({{J.skipped >= kMaxSkipped ? 0 : 1, work}, slot});
      }
    }
    std::sort(small.begin(), small.end());
    size_t g = 0, next = 0;
    if (!large_running && first_large >= 0) plan[g++].second.push_back(first_large);
    for (; g < plan.size() && next < small.size(); ++g) plan[g].second.push_back(small[next++].second);
  } else {
    std::vector<std::pair<std::pair<int, double>, int>> order;  // ((not forced, work), slot)
    for (int slot : cand) {
      const Job &J = job_at(slot);
      const double work = job_nodes(J) * double(std::max(0, J.spec.max_steps - J.steps));
      order.push_back({{J.skipped >= kMaxSkipped ? 0 : 1, work}, slot});
    }
    std::sort(order.begin(), order.end());
    const double fill = double(B->fill_nodes);
    size_t next = 0;
    for (size_t g = 0; g < plan.size() && next < order.size(); ++g) {
      std::vector<int> &grp = plan[g].second;
      double nodes = 0.0;
      // jobs left out too long all go into the first group
      while (g == 0 && next < order.size() && order[next].first.first == 0) {
        grp.push_back(order[next].second);
        nodes += job_nodes(job_at(order[next].second));
        ++next;
      }
      if (grp.empty()) {
        grp.push_back(order[next].second);
        nodes = job_nodes(job_at(order[next].second));
        ++next;
        if (nodes >= fill) continue;
      }
      while (next < order.size() && nodes < fill && job_nodes(job_at(order[next].second)) < fill) {
        grp.push_back(order[next].second);
        nodes += job_nodes(job_at(order[next].second));
        ++next;
      }
    }
  }
  std::vector<char> picked(size_t(B->max_jobs), 0);
  for (auto &p : plan) {
    std::sort(p.second.begin(), p.second.end());
    for (int slot : p.second) picked[slot] = 1;
  }
  for (int slot : cand) {
    Job &J = job_at(slot);
    J.skipped = picked[slot] ? 0 : J.skipped + 1;
  }
  plan.erase(std::remove_if(plan.begin(), plan.end(), [](const auto &p) { return p.second.empty(); }), plan.end());
  return plan;
}

// Enqueue one chunk of the jobs in `slots` on a lane: the steps, then the
// convergence measure and its copy to the host, then the lane's event.
lbm_status start_chunk(lbm_batch *B, int l, const std::vector<int> &slots) {
  Lane &ln = B->lanes[l];
  int running = 0;
  for (size_t o = 0; o < B->lanes.size(); ++o) {
    if (int(o) == l || !B->lanes[o].busy) continue;
    const hipError_t q = hipEventQuery(B->lanes[o].done);
    if (q == hipErrorNotReady)
      ++running;
    else if (q != hipSuccess)
      return bfail(LBM_ERR_HIP, "event query: %s", hipGetErrorString(q));
  }
  if (B->init_recorded) LBM_BHIP(hipStreamWaitEvent(ln.stream, B->init_done, 0), "wait for initialisation");
  lbm_status st = upload_tables(B, ln, slots);
  if (st != LBM_OK) return st;
  // one row-major job alone: the single-lattice sweep (population-major
  // rows that are not whole lines run faster in the batch's flat walk)
  const bool solo = slots.size() == 1 && B->jobs.at(B->slot_job[slots[0]]).layout == LBM_LAYOUT_ROW_MAJOR;
  // The convergence maxima start at zero (a fill kernel rather than a
  // memset: they are the bit patterns of non-negative floats, and 0.0f is
  // all zero bits); the chunk's last step takes the measure, or, when the
  // chunk ends with a pass of two steps, the measure kernel afterwards.
  const size_t nd = size_t(B->max_jobs);
  lbm::fill_float_kernel<<<dim3(unsigned((nd + 255) / 256)), dim3(256), 0, ln.stream>>>(
      reinterpret_cast<float *>(ln.d_delta), nd, 0.0f);
  LBM_BHIP(hipGetLastError(), "reset deltas");
  st = solo ? run_solo_chunk(B, ln, slots[0]) : run_graph_chunk(B, ln);
  if (st != LBM_OK) return st;
  // the measure: combined from the last step's per-wave maxima, or (after
  // a pass, or with persistent workgroups) taken from the state; persistent
  // workgroups, 8 per compute unit (a chunk of one job alone combined its
  // own in launch_sweep_delta)
  const bool measured = measured_in_last_step(B, solo);
  for (int s = 0; s < kNumStorage; ++s) {
    if (ln.ntiles[s] == 0 || (measured && solo)) continue;
    if (measured) {
      lbm::tile_partials_kernel<<<dim3(unsigned(8 * B->num_cu)), dim3(256), 0, ln.stream>>>(
          ln.d_tiles[s], ln.d_ntiles + s, ln.d_part + ln.part_off[s], B->shape.block_x / 64, ln.d_delta);
      LBM_BHIP(hipGetLastError(), "measure launch");
    } else {
      LBM_BHIP(lbm::launch_batch_delta(s, ln.d_lats, ln.d_tiles[s], ln.d_ntiles + s, ln.d_delta, 8 * B->num_cu,
                                       ln.stream),
               "measure launch");
    }
  }
  LBM_BHIP(hipMemcpyAsync(ln.h_delta.as<void>(), ln.d_delta, sizeof(unsigned) * nd, hipMemcpyDeviceToHost,
                          ln.stream),
           "copy deltas");
  LBM_BHIP(hipEventRecord(ln.done, ln.stream), "event");
  ln.busy = true;
  ln.slots = slots;
  for (int slot : slots) B->jobs.at(B->slot_job[slot]).lane = l;
  lbm_batch_stats &S = B->stats;
  ++S.chunks;
  S.job_chunks += (long long)slots.size();
  if (slots.size() >= 2) ++S.multi_job_chunks;
  S.max_jobs_in_chunk = std::max(S.max_jobs_in_chunk, int(slots.size()));
  if (running > 0) ++S.overlapped_chunks;
  S.max_lanes_running = std::max(S.max_lanes_running, running + 1);
  return LBM_OK;
}

// Results of a lane's completed chunk: step counts, convergence, retirement.
lbm_status finish_chunk(lbm_batch *B, int l) {
  Lane &ln = B->lanes[l];
  ln.busy = false;
  const unsigned *hd = ln.h_delta.as<unsigned>();
  for (int slot : ln.slots) {
    const int id = B->slot_job[slot];
    Job &J = B->jobs.at(id);
    J.lane = -1;
    J.steps += B->chunk_steps;
    float d;
    std::memcpy(&d, &hd[slot], sizeof(d));
    J.delta = d;
    const bool conv = J.spec.tol > 0.0 && J.delta < J.spec.tol;
    if (conv || J.steps >= J.spec.max_steps) {
      J.converged = conv ? 1 : 0;
      lbm_status st = retire(B, id, ln);
      if (st != LBM_OK) return st;
    }
  }
  ln.slots.clear();
  return LBM_OK;
}

// Block until at least one busy lane has completed its chunk; process every
// completed one.
lbm_status wait_and_finish(lbm_batch *B) {
  std::vector<int> busy;
  for (int l = 0; l < int(B->lanes.size()); ++l)
    if (B->lanes[l].busy) busy.push_back(l);
  if (busy.empty()) return LBM_OK;
  std::vector<int> ready;
  if (busy.size() == 1) {
    LBM_BHIP(hipEventSynchronize(B->lanes[busy[0]].done), "chunk");
    ready = busy;
  } else {
    for (;;) {
      for (int l : busy) {
        const hipError_t q = hipEventQuery(B->lanes[l].done);
        if (q == hipSuccess)
          ready.push_back(l);
        else if (q != hipErrorNotReady)
          return bfail(LBM_ERR_HIP, "chunk: %s", hipGetErrorString(q));
      }
      if (!ready.empty()) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  for (int l : ready) {
    lbm_status st = finish_chunk(B, l);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

lbm_status drain(lbm_batch *B) {
  for (;;) {
    bool any = false;
    for (const Lane &ln : B->lanes) any = any || ln.busy;
    if (!any) return LBM_OK;
    lbm_status st = wait_and_finish(B);
    if (st != LBM_OK) return st;
  }
}

int count_active(const lbm_batch *B) {
  int n = 0;
  for (int id : B->slot_job) n += id >= 0;
  return n;
}

long long tune_key(const lbm_batch *B, const Lane &ln) {
  size_t nodes = 0;
  for (int id : B->slot_job)
    if (id >= 0) nodes += B->jobs.at(id).nodes;
  int lg = 0;
  while ((size_t(1) << lg) < nodes) ++lg;
  return (long long)present_mask(ln) | ((long long)lg << 4) | ((long long)B->pass_steps << 12);
}

}  // namespace

extern "C" {

lbm_status lbm_job_bytes(const lbm_job *job, size_t *bytes) {
  if (!job || !bytes) return bfail(LBM_ERR_ARG, "NULL argument");
  if (lbm_element_bytes(job->storage) == 0) return bfail(LBM_ERR_ARG, "invalid storage");
  // either layout a batch may give the job
  *bytes = std::max(job_bytes(*job, LBM_LAYOUT_ROW_MAJOR),
                    job_bytes(*job, batch_layout_kind(job->nx, lbm_element_bytes(job->storage))));
  return LBM_OK;
}

lbm_status lbm_batch_create(size_t hbm_budget_bytes, int chunk_steps, int max_jobs, void *hip_stream,
                            lbm_batch **out) {
  if (!out) return bfail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (chunk_steps < 2 || chunk_steps % 2) return bfail(LBM_ERR_ARG, "chunk_steps must be even and >= 2");
  if (max_jobs < 1 || max_jobs > 65536) return bfail(LBM_ERR_ARG, "max_jobs must be in [1, 65536]");
  if (hbm_budget_bytes < (size_t(1) << 20)) return bfail(LBM_ERR_ARG, "HBM budget below 1 MiB");
  lbm_batch *B = new (std::nothrow) lbm_batch();
  if (!B) return bfail(LBM_ERR_OOM, "host allocation failed");
  B->chunk_steps = chunk_steps;
  B->max_jobs = max_jobs;
  B->user_stream = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    B->num_cu = prop.multiProcessorCount;
  B->stats.lanes = 1;
  B->lanes.resize(1);
  lbm_status st = init_lane(B, B->lanes[0], B->user_stream);
  if (st == LBM_OK && (hipStreamCreateWithFlags(&B->init_stream, hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreateWithFlags(&B->init_done, hipEventDisableTiming) != hipSuccess)) {
    (void)hipGetLastError();
    st = bfail(LBM_ERR_HIP, "stream or event creation failed");
  }
  if (st != LBM_OK) {
    lbm_batch_destroy(B);
    return st;
  }
  const size_t cap = hbm_budget_bytes / kAlign * kAlign;
  hipError_t e = hipMalloc(&B->pool_base, cap);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    lbm_batch_destroy(B);
    return bfail(LBM_ERR_OOM, "hipMalloc of the %zu-byte pool failed: %s", cap, hipGetErrorString(e));
  }
  B->pool.reset(cap);
  B->slot_job.assign(max_jobs, -1);
  B->lat.assign(max_jobs, lbm::BatchLat());
  std::memset(B->lat.data(), 0, B->lat.size() * sizeof(lbm::BatchLat));
  *out = B;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *B) {
  if (!B) return;
  for (Lane &ln : B->lanes) free_lane(ln);
  if (B->init_stream) (void)hipStreamSynchronize(B->init_stream);
  if (B->init_done) (void)hipEventDestroy(B->init_done);
  if (B->init_stream) (void)hipStreamDestroy(B->init_stream);
  if (B->pool_base) (void)hipFree(B->pool_base);
  delete B;
}

lbm_status lbm_batch_set_lanes(lbm_batch *B, int lanes) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  if (lanes < 1 || lanes > kMaxLanes) return bfail(LBM_ERR_ARG, "lanes must be in [1, %d] (got %d)", kMaxLanes, lanes);
  for (const Lane &ln : B->lanes)
    if (ln.busy) return bfail(LBM_ERR_STATE, "a chunk is in flight");
  for (int id : B->slot_job)
    if (id >= 0 && B->jobs.at(id).lane >= 0) return bfail(LBM_ERR_STATE, "a chunk is in flight");
  while (int(B->lanes.size()) > lanes) {
    free_lane(B->lanes.back());
    B->lanes.pop_back();
  }
  while (int(B->lanes.size()) < lanes) {
    B->lanes.emplace_back();
    lbm_status st = init_lane(B, B->lanes.back(), nullptr);
    if (st != LBM_OK) {
      free_lane(B->lanes.back());
      B->lanes.pop_back();
      return st;
    }
  }
  B->stats.lanes = lanes;
  return LBM_OK;
}

lbm_status lbm_batch_submit(lbm_batch *B, const lbm_job *job, int *job_id) {
  if (!B || !job || !job_id) return bfail(LBM_ERR_ARG, "NULL argument");
  const lbm_job &j = *job;
  if (j.nx < 1 || j.ny < 1 || j.nz < 1) return bfail(LBM_ERR_ARG, "lattice sizes must be >= 1");
  if (double(j.nx) * j.ny * j.nz >= 2147483648.0) return bfail(LBM_ERR_ARG, "at most 2^31 - 1 nodes");
  if (!(j.tau > 0.5)) return bfail(LBM_ERR_ARG, "tau must be > 1/2");
  if (!(j.rho0 > 0.0)) return bfail(LBM_ERR_ARG, "rho0 must be > 0");
  if (lbm_element_bytes(j.storage) == 0) return bfail(LBM_ERR_ARG, "invalid storage");
  if (!(j.u_ref > 0.0)) return bfail(LBM_ERR_ARG, "u_ref must be > 0");
  if (double(lbm::buffer_elements(LBM_LAYOUT_ROW_MAJOR, j.nx, j.ny, j.nz, lbm_element_bytes(j.storage))) *
          double(lbm_element_bytes(j.storage)) >= 4294967296.0 ||
      19.0 * double(lbm::population_pitch(size_t(j.nx) * j.ny * j.nz)) * double(lbm_element_bytes(j.storage)) >=
          4294967296.0)
    return bfail(LBM_ERR_ARG, "a batch job's population buffer must stay below 4 GiB (19 N element bytes, rows padded)");
  if (j.max_steps < 0) return bfail(LBM_ERR_ARG, "max_steps must be >= 0");
  if (j.bc_mask & ~63u) return bfail(LBM_ERR_ARG, "bc_mask has bits beyond the six faces");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(j.force[d])) return bfail(LBM_ERR_ARG, "force is not finite");
  const int size[3] = {j.nx, j.ny, j.nz};
  if (j.pressure_mask & ~j.bc_mask) return bfail(LBM_ERR_ARG, "pressure_mask must be a subset of bc_mask");
  int p_axes = 0;
  for (int a = 0; a < 3; ++a) {
    const unsigned bits = (j.bc_mask >> (2 * a)) & 3u;
    if (bits == 1u || bits == 2u) return bfail(LBM_ERR_ARG, "axis %d has a BC on one face only", a);
    if (bits && size[a] < 3) return bfail(LBM_ERR_ARG, "a bounded axis needs at least 3 nodes");
    p_axes += ((j.pressure_mask >> (2 * a)) & 3u) != 0u;
  }
  if (p_axes > 1) return bfail(LBM_ERR_ARG, "pressure faces must lie on one axis");
  for (int f = 0; f < 6; ++f) {
    if (!((j.bc_mask >> f) & 1u)) continue;
    const double *u = j.bc_velocity[f];
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(u[d])) return bfail(LBM_ERR_ARG, "face %d velocity is not finite", f);
    const double un = u[0] * lbm::kFaceNormal[f][0] + u[1] * lbm::kFaceNormal[f][1] + u[2] * lbm::kFaceNormal[f][2];
    if ((j.pressure_mask >> f) & 1u) {
      if (!std::isfinite(j.bc_rho[f]) || !(j.bc_rho[f] > 0.0))
        return bfail(LBM_ERR_ARG, "face %d density must be a positive finite number", f);
      if (!(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] - un * un < 1.0 / 3.0))
        return bfail(LBM_ERR_ARG, "face %d tangential velocity out of range (|u_t| < 1/sqrt(3) required)", f);
      continue;
    }
    if (!(std::fabs(un) < 1.0) || !(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] < 1.0 / 3.0))
      return bfail(LBM_ERR_ARG, "face %d velocity out of range (|u.n| < 1 and |u| < 1/sqrt(3) required)", f);
  }
  Job J;
  J.spec = j;
  J.nodes = size_t(j.nx) * j.ny * j.nz;
  // The layout is fixed here: row-major with padded rows for every job with
  // two steps per pass (the pass's tiles are rows of one population) and
  // for a job that every chunk steps alone through the single-lattice sweep
  // (shortest first, at least fill_nodes nodes), else row-major only for
  // rows of whole 128-byte lines.
  const bool alone = B->policy == LBM_BATCH_LARGE_IN_ORDER ||
                     (B->policy == LBM_BATCH_SHORTEST_FIRST && double(J.nodes) >= double(B->fill_nodes));
  J.layout = (alone || B->pass_steps == 2) ? LBM_LAYOUT_ROW_MAJOR
                                           : batch_layout_kind(j.nx, lbm_element_bytes(j.storage));
  J.bytes = job_bytes(j, J.layout);
  if (J.bytes > B->pool.capacity())
    return bfail(LBM_ERR_OOM, "job needs %zu bytes, more than the whole budget (%zu)", J.bytes, B->pool.capacity());
  const int id = B->next_id++;
  B->jobs.emplace(id, std::move(J));
  B->queue.push_back(id);
  *job_id = id;
  return LBM_OK;
}

lbm_status lbm_batch_run_chunk(lbm_batch *B, int *n_active, int *n_queued) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  lbm_status st = admit(B);
  if (st != LBM_OK) return st;
  for (const auto &p : plan_chunks(B)) {
    st = start_chunk(B, p.first, p.second);
    if (st != LBM_OK) return st;
  }
  st = wait_and_finish(B);
  if (st != LBM_OK) return st;
  if (n_active) *n_active = count_active(B);
  if (n_queued) *n_queued = int(B->queue.size());
  return LBM_OK;
}

lbm_status lbm_batch_poll(lbm_batch *B, int job_id, lbm_job_status *st) {
  if (!B || !st) return bfail(LBM_ERR_ARG, "NULL argument");
  auto it = B->jobs.find(job_id);
  if (it == B->jobs.end()) return bfail(LBM_ERR_ARG, "unknown job %d", job_id);
  st->state = it->second.state;
  st->steps = it->second.steps;
  st->delta = it->second.delta;
  st->converged = it->second.converged;
  st->nodes = (long long)it->second.nodes;
  return LBM_OK;
}

lbm_status lbm_batch_result(lbm_batch *B, int job_id, double *rho, double *u) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  auto it = B->jobs.find(job_id);
  if (it == B->jobs.end()) return bfail(LBM_ERR_ARG, "unknown job %d", job_id);
  if (it->second.state != LBM_JOB_DONE) return bfail(LBM_ERR_STATE, "job %d is not finished", job_id);
  const size_t N = it->second.nodes;
  const double *r = it->second.result.as<double>();
  if (rho) std::memcpy(rho, r, N * sizeof(double));
  if (u) std::memcpy(u, r + N, 3 * N * sizeof(double));
  give_back_result_block(B, std::move(it->second.result));
  B->jobs.erase(it);
  return LBM_OK;
}

lbm_status lbm_batch_set_shape(lbm_batch *B, int block_x, int tile_nodes, int grid_blocks) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  if (block_x != 128 && block_x != 256) return bfail(LBM_ERR_ARG, "block_x must be 128 or 256");
  if (tile_nodes < kMinTileNodes) return bfail(LBM_ERR_ARG, "tile_nodes must be >= %d", kMinTileNodes);
  if (grid_blocks < 0 || grid_blocks > (1 << 20)) return bfail(LBM_ERR_ARG, "grid_blocks out of range");
  for (const Lane &ln : B->lanes)
    if (ln.busy) return bfail(LBM_ERR_STATE, "a chunk is in flight");
  if (B->shape.block_x != block_x || B->shape.grid != grid_blocks)
    for (Lane &ln : B->lanes) drop_graphs(ln);
  B->shape.block_x = block_x;
  B->shape.tile_nodes = tile_nodes;
  B->shape.grid = grid_blocks;
  return LBM_OK;
}

lbm_status lbm_batch_set_steps_per_pass(lbm_batch *B, int steps_per_pass, int z_planes) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  if (steps_per_pass != 1 && steps_per_pass != 2)
    return bfail(LBM_ERR_ARG, "steps_per_pass must be 1 or 2 (got %d)", steps_per_pass);
  if (z_planes < 0 || z_planes > 4096) return bfail(LBM_ERR_ARG, "z_planes must be in [0, 4096] (got %d)", z_planes);
  for (const Lane &ln : B->lanes)
    if (ln.busy) return bfail(LBM_ERR_STATE, "a chunk is in flight");
  if (steps_per_pass == 2)
    for (const auto &kv : B->jobs)
      if ((kv.second.state == LBM_JOB_QUEUED || kv.second.state == LBM_JOB_RUNNING) &&
          kv.second.layout != LBM_LAYOUT_ROW_MAJOR)
        return bfail(LBM_ERR_STATE, "job %d is stored population-major: two steps per pass need row-major jobs "
                     "(set the mode before submitting)", kv.first);
  B->pass_steps = steps_per_pass;
  B->pass_zc = z_planes == 0 ? 32 : z_planes;
  return LBM_OK;
}

lbm_status lbm_batch_get_steps_per_pass(const lbm_batch *B, int *steps_per_pass, int *z_planes) {
  if (!B || !steps_per_pass || !z_planes) return bfail(LBM_ERR_ARG, "NULL argument");
  *steps_per_pass = B->pass_steps;
  *z_planes = B->pass_zc;
  return LBM_OK;
}

lbm_status lbm_batch_set_policy(lbm_batch *B, int policy, size_t fill_nodes) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  if (policy != LBM_BATCH_LOCKSTEP && policy != LBM_BATCH_SHORTEST_FIRST && policy != LBM_BATCH_LARGE_IN_ORDER)
    return bfail(LBM_ERR_ARG,
                 "policy must be LBM_BATCH_LOCKSTEP, LBM_BATCH_SHORTEST_FIRST or LBM_BATCH_LARGE_IN_ORDER (got %d)",
                 policy);
  B->policy = policy;
  B->fill_nodes = fill_nodes;
  return LBM_OK;
}

lbm_status lbm_batch_get_shape(const lbm_batch *B, int *block_x, int *tile_nodes, int *grid_blocks) {
  if (!B || !block_x || !tile_nodes || !grid_blocks) return bfail(LBM_ERR_ARG, "NULL argument");
  *block_x = B->shape.block_x;
  *tile_nodes = B->shape.tile_nodes;
  *grid_blocks = B->shape.grid;
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *B, int trial_steps, int *block_x, int *tile_nodes, int *grid_blocks) {
  if (!B) return bfail(LBM_ERR_ARG, "NULL handle");
  if (trial_steps < 2 || trial_steps % 2) return bfail(LBM_ERR_ARG, "trial_steps must be even and >= 2");
  lbm_status st = drain(B);
  if (st != LBM_OK) return st;
  st = admit(B);
  if (st != LBM_OK) return st;
  if (count_active(B) == 0) return bfail(LBM_ERR_STATE, "no resident job to tune on");
  // trial steps are steps of every resident job, on lane 0
  Lane &ln = B->lanes[0];
  if (B->init_recorded) LBM_BHIP(hipStreamWaitEvent(ln.stream, B->init_done, 0), "wait for initialisation");
  std::vector<int> all;
  for (int slot = 0; slot < B->max_jobs; ++slot)
    if (B->slot_job[slot] >= 0) all.push_back(slot);
  st = upload_tables(B, ln, all);
  if (st != LBM_OK) return st;
  const long long key = tune_key(B, ln);
  Tuned cached;
  bool have_cached = false;
  {
    std::lock_guard<std::mutex> lock(g_tuned_mutex);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      cached = it->second;
      have_cached = true;
    }
  }
  const bool pass2 = B->pass_steps == 2;
  if (have_cached) {
    st = lbm_batch_set_shape(B, cached.shape.block_x, cached.shape.tile_nodes, cached.shape.grid);
    B->pass_zc = cached.zc;
    B->pass_remap = cached.remap;
  } else {
    // Every trial step is a real step of every resident lattice (results do
    // not depend on the launch shape); the step counters advance with them.
    // With two steps per pass the candidates are the pass's z ranges and box
    // orders (the single step's shape stays the default: chunks of a
    // multiple of 4 steps take no single step), timed over at least 4 steps
    // (2 passes), a multiple of 4, after 2 warm-up passes.
    const int warm = pass2 ? 4 : 2;
    const int timed = pass2 ? (std::max(trial_steps, 4) + 3) / 4 * 4 : trial_steps;
    std::vector<Tuned> cands;
    if (pass2) {
      for (int zc : {16, 32, 64})
        for (int remap : {1, 0}) cands.push_back({Shape(), zc, remap});
    } else {
      // one workgroup per tile of 256-1024 nodes, and two persistent grids
      for (const Shape &c : {Shape{256, 256, 0}, Shape{256, 512, 0}, Shape{256, 1024, 0}, Shape{128, 256, 0},
                             Shape{256, 1024, 16 * B->num_cu}, Shape{128, 1024, 8 * B->num_cu}})
        cands.push_back({c, B->pass_zc, B->pass_remap});
    }
    hipEvent_t e0, e1;
    LBM_BHIP(hipEventCreate(&e0), "event");
    LBM_BHIP(hipEventCreate(&e1), "event");
    Tuned best;
    float best_ms = INFINITY;
    for (const Tuned &c : cands) {
      st = lbm_batch_set_shape(B, c.shape.block_x, c.shape.tile_nodes, c.shape.grid);
      B->pass_zc = c.zc;
      B->pass_remap = c.remap;
      if (st == LBM_OK) st = upload_tables(B, ln, all);
      if (st == LBM_OK) st = launch_steps(B, ln, warm, 0, false);
      hipError_t e = st == LBM_OK ? hipEventRecord(e0, ln.stream) : hipSuccess;
      if (st == LBM_OK && e == hipSuccess) st = launch_steps(B, ln, timed, warm, false);
      if (st == LBM_OK && e == hipSuccess) e = hipEventRecord(e1, ln.stream);
      if (st == LBM_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (st == LBM_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (st != LBM_OK || e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return st != LBM_OK ? st : bfail(LBM_ERR_HIP, "autotune timing: %s", hipGetErrorString(e));
      }
      for (int slot : all) B->jobs.at(B->slot_job[slot]).steps += warm + timed;
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
      std::lock_guard<std::mutex> lock(g_tuned_mutex);
      g_tuned[key] = best;
    }
    st = lbm_batch_set_shape(B, best.shape.block_x, best.shape.tile_nodes, best.shape.grid);
    B->pass_zc = best.zc;
    B->pass_remap = best.remap;
  }
  if (st != LBM_OK) return st;
  if (block_x) *block_x = B->shape.block_x;
  if (tile_nodes) *tile_nodes = B->shape.tile_nodes;
  if (grid_blocks) *grid_blocks = B->shape.grid;
  return LBM_OK;
}

lbm_status lbm_batch_memory(const lbm_batch *B, size_t *used, size_t *capacity) {
  if (!B || !used || !capacity) return bfail(LBM_ERR_ARG, "NULL argument");
  *used = B->pool.used();
  *capacity = B->pool.capacity();
  return LBM_OK;
}

lbm_status lbm_batch_get_stats(const lbm_batch *B, lbm_batch_stats *stats) {
  if (!B || !stats) return bfail(LBM_ERR_ARG, "NULL argument");
  *stats = B->stats;
  return LBM_OK;
}

}  // extern "C"
