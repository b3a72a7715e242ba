// lbm_kernels.hip -- HIP kernels for gfx950: the fused D3Q19 sweep (pull
// streaming + on-site boundary rules + BGK), initialisation, moments and
// FP64 reductions, storage conversion and bandwidth probes.
//
// Layout in HBM (PopLayout): population-major, population k of node n at
// k*P + n, n = x + nx*(y + ny*z), P = N rounded up to a multiple of 64
// (population starts on cache-line boundaries); or row-major, the 19
// populations of each x-row next to each other (element k*nx + 19*nx*r + x
// for row r = y + ny*z).  One sweep reads 19 and writes 19 elements per node;
// every element of the source buffer is read exactly once per step (the pull
// scheme has no reuse between nodes), so the kernel is a pure 38-stream HBM
// copy with ~200 flops per node on top.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "d3q19.hpp"
#include "lbm_internal.hpp"
#include "node_update.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// The fused sweep over one lattice.  One block handles BX*NPT consecutive
// nodes of one x-row; thread t handles x = x0 + j*BX + t, j < NPT (coalesced
// 64-lane accesses).  y and z are uniform over the block, so the row offsets
// of the nine source rows are scalar and each load is "scalar base + lane
// offset".  COPY: streaming only (no boundary rule, no collision, raw
// elements) -- the bandwidth ceiling of this access pattern.  EXT: the
// extended update with solid nodes and per-node face velocities (a.ext).
// ROWS: the row-major layout through per-row buffer descriptors (RowAccess;
// the row of a solid node's own populations is per lane, so not with EXT);
// otherwise plain pointers.  Stores are non-temporal either way: the
// destination is not read again before the next step, which streams through
// far more data than the caches hold.
// ---------------------------------------------------------------------------
template <class F, int BX, int NPT, bool ROWS, bool COPY, bool EXT>
__global__ __launch_bounds__(BX) void sweep_kernel(const typename F::S *__restrict__ src,
                                                   typename F::S *__restrict__ dst,
                                                   SweepArgs<typename Codec<typename F::S>::T> a) {
  static_assert(!(ROWS && EXT), "per-row descriptors need a wave-uniform row");
  using S = typename F::S;
  const unsigned b = logical_block(blockIdx.x, gridDim.x, a.xcd_remap, unsigned(a.nxc));
  const unsigned row = a.nxc == 1 ? b : b / unsigned(a.nxc);
  const int xc = int(b - row * unsigned(a.nxc));
  const NodeGeom g{unsigned(a.nx), unsigned(a.ny), unsigned(a.nz), a.row_stride};
  using Access = std::conditional_t<ROWS, RowAccess<S>, PtrAccess<S, true>>;
  Access mem;
  if constexpr (ROWS)
    mem = Access{src, dst, unsigned(a.pop_stride * sizeof(S)), unsigned(a.row_stride * sizeof(S))};
  else
    mem = Access{src, dst, a.pop_stride};
  const int y = int(row % g.ny);
  const int z = int(row / g.ny);
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int x = (xc * NPT + j) * BX + int(threadIdx.x);
    if (x < a.nx) update_node<F, COPY, EXT>(mem, g, x, y, z, a.p, a.key, a.ext);
  }
}

// The sweep that ends a chunk of the batch runtime for a job stepped alone:
// sweep_kernel's update (one node per thread, non-temporal stores), and the
// convergence measure of the state it writes (velocity_change): each wave's
// maximum goes to partials[block * BX / 64 + wave], with a plain store (one
// atomic per wave on one address, across the XCDs' separate L2 caches, made
// the step 3.6 times slower).
template <class F, int BX>
__global__ __launch_bounds__(BX) void sweep_delta_kernel(const typename F::S *__restrict__ src,
                                                         typename F::S *__restrict__ dst,
                                                         SweepArgs<typename Codec<typename F::S>::T> a, DeltaArgs dl,
                                                         float *__restrict__ partials) {
  using S = typename F::S;
  using T = typename Codec<S>::T;
  const unsigned b = logical_block(blockIdx.x, gridDim.x, a.xcd_remap, unsigned(a.nxc));
  const unsigned row = a.nxc == 1 ? b : b / unsigned(a.nxc);
  const int xc = int(b - row * unsigned(a.nxc));
  const NodeGeom g{unsigned(a.nx), unsigned(a.ny), unsigned(a.nz), a.row_stride};
  const PtrAccess<S, true> mem{src, dst, a.pop_stride};
  const int y = int(row % g.ny);
  const int z = int(row / g.ny);
  const int x = xc * BX + int(threadIdx.x);
  float dmax = 0.0f;
  if (x < a.nx)
    update_node<F, false, false, T, PtrAccess<S, true>, true>(mem, g, x, y, z, a.p, a.key, a.ext, dl, &dmax);
  dmax = wave_max(dmax);
  if ((threadIdx.x & 63) == 0) partials[size_t(blockIdx.x) * (BX / 64) + (threadIdx.x >> 6)] = dmax;
}

// Maximum of partials[0 .. count) into *delta_bits (the bit pattern of a
// non-negative float; *delta_bits starts at zero): workgroups of 256
// threads stride over the partials, one atomic maximum each (a single
// workgroup took 0.37 ms over the 262144 partials of a 256^3 lattice).
__global__ __launch_bounds__(256) void max_partials_kernel(const float *__restrict__ partials, size_t count,
                                                           unsigned *__restrict__ delta_bits) {
  __shared__ float lds[4];
  float m = 0.0f;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256)
    m = fmaxf(m, partials[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(delta_bits, __float_as_uint(fmaxf(fmaxf(lds[0], lds[1]), fmaxf(lds[2], lds[3]))));
}

// ---------------------------------------------------------------------------
// Initialisation: f_k = f_k^eq(rho0, u0) at every node (eq_feq), stored as
// d_k = f_k - w_k = w_k (rho0 - 1) + w_k rho0 (3 c.u + 4.5 (c.u)^2 - 1.5 u^2),
// evaluated in double.
// ---------------------------------------------------------------------------
template <class S>
__global__ void init_kernel(S *__restrict__ f, size_t N, PopLayout lay, double rho0, double ux, double uy,
                            double uz) {
  const size_t n = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const size_t at = lay.index(0, n);
  const double usq15 = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const double cu = double(cx(k)) * ux + double(cy(k)) * uy + double(cz(k)) * uz;
    const double dk = weight<double>(k) * ((rho0 - 1.0) + rho0 * (3.0 * cu + 4.5 * cu * cu - usq15));
    f[at + size_t(k) * lay.pop_stride] = Codec<S>::encode(typename Codec<S>::T(dk));
  }
}

// ---------------------------------------------------------------------------
// Moments of the stored state (eq_rho, eq_vel) for nodes [n0, n0 + count):
// rho = 1 + sum_k d_k and rho u = sum_k d_k c_k (the weights sum to 1 and have
// zero first moment); rho[i], u[a*count + i] in double; optional per-block FP64 partial sums of
// mass and momentum (wavefront shuffles, then LDS across the block's waves,
// in a fixed order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <class S>
__global__ __launch_bounds__(256) void moments_kernel(const S *__restrict__ f, PopLayout lay, size_t n0,
                                                      size_t count, double *__restrict__ rho,
                                                      double *__restrict__ u,
                                                      double *__restrict__ partials) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride) {
    const size_t at = lay.index(0, n0 + i);
    double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const double v = double(Codec<S>::decode(f[at + size_t(k) * lay.pop_stride]));
      dr += v;
      if (cx(k)) jx += double(cx(k)) * v;
      if (cy(k)) jy += double(cy(k)) * v;
      if (cz(k)) jz += double(cz(k)) * v;
    }
    const double r = 1.0 + dr;
    if (rho) rho[i] = r;
    if (u) {
      u[i] = jx / r;
      u[count + i] = jy / r;
      u[2 * count + i] = jz / r;
    }
    acc[0] += r;
    acc[1] += jx;
    acc[2] += jy;
    acc[3] += jz;
  }
  if (!partials) return;
  __shared__ double lds[4][4];  // [wave][quantity], blockDim = 256 = 4 waves
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double s = wave_sum(acc[c]);
    if (lane == 0) lds[wave][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    partials[size_t(blockIdx.x) * 4 + c] = ((lds[0][c] + lds[1][c]) + lds[2][c]) + lds[3][c];
  }
}

// Final fixed-order reduction of nblk partial quadruples into out[4].
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *__restrict__ partials, int nblk,
                                                              double *__restrict__ out) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += partials[size_t(b) * 4 + c];
  __shared__ double lds[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double s = wave_sum(acc[c]);
    if (lane == 0) lds[wave][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    out[c] = ((lds[0][c] + lds[1][c]) + lds[2][c]) + lds[3][c];
  }
}

// ---------------------------------------------------------------------------
// Conversion between the stored form and populations f_k = w_k + d_k in
// double, nodes [n0, n0 + count); the chunk's layout is buf[k*count + i].
// ---------------------------------------------------------------------------
template <class S>
__global__ void to_double_kernel(const S *__restrict__ f, PopLayout lay, size_t n0, size_t count,
                                 double *__restrict__ out) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const size_t at = lay.index(0, n0 + i);
#pragma unroll
  for (int k = 0; k < 19; ++k)
    out[size_t(k) * count + i] =
        weight<double>(k) + double(Codec<S>::decode(f[at + size_t(k) * lay.pop_stride]));
}

template <class S>
__global__ void from_double_kernel(S *__restrict__ f, PopLayout lay, size_t n0, size_t count,
                                   const double *__restrict__ in) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const size_t at = lay.index(0, n0 + i);
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    using T = typename Codec<S>::T;
    f[at + size_t(k) * lay.pop_stride] = Codec<S>::encode(T(in[size_t(k) * count + i] - weight<double>(k)));
  }
}

// Raw element copy of a state from one layout into another (no arithmetic:
// the stored encodings move unchanged).
template <class E>
__global__ void relayout_kernel(const E *__restrict__ src, PopLayout from, E *__restrict__ dst, PopLayout to,
                                size_t N) {
  const size_t n = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const size_t a = from.index(0, n), b = to.index(0, n);
#pragma unroll
  for (int k = 0; k < 19; ++k) dst[b + size_t(k) * to.pop_stride] = src[a + size_t(k) * from.pop_stride];
}

// Plain contiguous copy of nbytes (multiple of 16): one 16-byte element per
// thread, the form of the fastest read/write stream measured on the MI355X
// (the ceiling a 50/50 read/write kernel can reach on the device).
__global__ __launch_bounds__(256) void copy_probe_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                         size_t n16) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <class F, int BX, int NPT, bool ROWS, bool COPY, bool EXT>
static hipError_t launch_sweep_t(const void *src, void *dst, const SweepArgs<typename Codec<typename F::S>::T> &a,
                                 hipStream_t s) {
  using S = typename F::S;
  sweep_kernel<F, BX, NPT, ROWS, COPY, EXT><<<dim3(a.nblocks), dim3(BX), 0, s>>>(static_cast<const S *>(src),
                                                                              static_cast<S *>(dst), a);
  return hipGetLastError();
}

template <class F, bool ROWS, bool COPY>
static hipError_t launch_sweep_shape_t(const void *src, void *dst,
                                       const SweepArgs<typename Codec<typename F::S>::T> &a, int bx, int npt,
                                       hipStream_t s) {
#define LBM_CASE(B, P) \
  if (bx == B && npt == P) return launch_sweep_t<F, B, P, ROWS, COPY, false>(src, dst, a, s);
  LBM_CASE(64, 1) LBM_CASE(64, 2) LBM_CASE(64, 4)
  LBM_CASE(128, 1) LBM_CASE(128, 2) LBM_CASE(128, 4)
  LBM_CASE(256, 1) LBM_CASE(256, 2) LBM_CASE(256, 4)
  LBM_CASE(512, 1) LBM_CASE(512, 2) LBM_CASE(512, 4)
#undef LBM_CASE
  return hipErrorInvalidValue;
}

template <class F, bool COPY>
static hipError_t launch_sweep_shape(const void *src, void *dst,
                                     const SweepArgs<typename Codec<typename F::S>::T> &a, int bx, int npt,
                                     hipStream_t s) {
  // The row-major layout (one row holds all 19 populations) through per-row
  // descriptors while a row's bytes fit their 31-bit offsets, for the FP16
  // and FP64 forms.  Measured per step on a 512x256x256 duct, both forms in turn on one device,
  // against plain pointers: FP16 round-to-nearest 0.445 against 0.453 ms,
  // FP64 1.752 against 1.769 ms, FP16 with stochastic rounding equal
  // (0.446 / 0.444: its vector instructions fell from about 424 to 348 per
  // node without a gain, so the sweep is bound by memory, not issue), FP32
  // 0.894 against 0.888 ms -- so FP32 keeps the pointers.
  if constexpr (sizeof(typename F::S) != 4) {
    const bool rows =
        a.row_stride >= 19 * a.pop_stride && a.row_stride * sizeof(typename F::S) < (size_t(1) << 31);
    if (rows) return launch_sweep_shape_t<F, true, COPY>(src, dst, a, bx, npt, s);
  }
  return launch_sweep_shape_t<F, false, COPY>(src, dst, a, bx, npt, s);
}

// The extended sweep runs one node per thread.
template <class F>
static hipError_t launch_sweep_ext(const void *src, void *dst, const SweepArgs<typename Codec<typename F::S>::T> &a,
                                   int bx, hipStream_t s) {
  switch (bx) {
    case 64: return launch_sweep_t<F, 64, 1, false, false, true>(src, dst, a, s);
    case 128: return launch_sweep_t<F, 128, 1, false, false, true>(src, dst, a, s);
    case 256: return launch_sweep_t<F, 256, 1, false, false, true>(src, dst, a, s);
    case 512: return launch_sweep_t<F, 512, 1, false, false, true>(src, dst, a, s);
  }
  return hipErrorInvalidValue;
}

template <class T>
static SweepArgs<T> make_args(const SweepConfig &c) {
  SweepArgs<T> a;
  a.nx = c.nx;
  a.ny = c.ny;
  a.nz = c.nz;
  a.pop_stride = c.layout.pop_stride;
  a.row_stride = c.layout.row_stride;
  const int span = c.block_x * c.nodes_per_thread;
  a.nxc = (c.nx + span - 1) / span;
  a.nblocks = unsigned(a.nxc) * unsigned(c.ny) * unsigned(c.nz);
  a.xcd_remap = c.xcd_remap;
  a.p.bc_mask = c.bc_mask;
  a.p.p_mask = c.p_mask;
  a.p.rule_flags = c.rule_flags;
  a.ext.solid = c.solid;
  a.ext.code = c.geo_code;
  for (int f = 0; f < 6; ++f) a.ext.face_v[f] = c.face_v[f];
  for (int f = 0; f < 6; ++f) a.p.rho_p[f] = T(c.rho_p[f]);
  a.p.omega = T(1.0 / c.tau);
  for (int d = 0; d < 3; ++d) a.p.tau_f[d] = T(c.tau * c.force[d]);
  a.key = step_key(c.step);
  for (int f = 0; f < 6; ++f)
    for (int d = 0; d < 3; ++d) a.p.fv.v[f][d] = T(c.v[f][d]);
  return a;
}

template <class F>
static hipError_t launch_sweep_delta_t(const SweepConfig &c, const void *src, void *dst, const DeltaArgs &dl,
                                       float *partials, hipStream_t s) {
  using S = typename F::S;
  const auto a = make_args<typename Codec<S>::T>(c);
  const S *in = static_cast<const S *>(src);
  S *out = static_cast<S *>(dst);
  switch (c.block_x) {
    case 64: sweep_delta_kernel<F, 64><<<dim3(a.nblocks), dim3(64), 0, s>>>(in, out, a, dl, partials); break;
    case 128: sweep_delta_kernel<F, 128><<<dim3(a.nblocks), dim3(128), 0, s>>>(in, out, a, dl, partials); break;
    case 256: sweep_delta_kernel<F, 256><<<dim3(a.nblocks), dim3(256), 0, s>>>(in, out, a, dl, partials); break;
    case 512: sweep_delta_kernel<F, 512><<<dim3(a.nblocks), dim3(512), 0, s>>>(in, out, a, dl, partials); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t sweep_delta_partials(const SweepConfig &c) {
  const size_t nxc = (size_t(c.nx) + size_t(c.block_x) - 1) / size_t(c.block_x);
  return nxc * size_t(c.ny) * size_t(c.nz) * size_t(c.block_x / 64);
}

hipError_t launch_sweep_delta(const SweepConfig &c_in, const void *src, void *dst, float *snap, double inv_uref,
                              float *partials, unsigned *delta_bits, hipStream_t s) {
  SweepConfig c = c_in;
  bool ext = c.solid != nullptr || c.geo_code != nullptr;
  for (int f = 0; f < 6; ++f) ext = ext || c.face_v[f] != nullptr;
  if (ext || c.block_x < 64) return hipErrorInvalidValue;
  c.nodes_per_thread = 1;
  const DeltaArgs dl{(global_ptr<float>)snap, size_t(c.nx) * size_t(c.ny) * size_t(c.nz), inv_uref};
  hipError_t e = hipErrorInvalidValue;
  switch (c.storage) {
    case kStoreF64: e = launch_sweep_delta_t<FormF64>(c, src, dst, dl, partials, s); break;
    case kStoreF32: e = launch_sweep_delta_t<FormF32>(c, src, dst, dl, partials, s); break;
    case kStoreF16: e = launch_sweep_delta_t<FormF16>(c, src, dst, dl, partials, s); break;
    case kStoreF16SR: e = launch_sweep_delta_t<FormF16SR>(c, src, dst, dl, partials, s); break;
  }
  if (e != hipSuccess) return e;
  const size_t np = sweep_delta_partials(c);
  const unsigned grid = unsigned(std::min<size_t>(64, (np + 4095) / 4096));
  max_partials_kernel<<<dim3(grid), dim3(256), 0, s>>>(partials, np, delta_bits);
  return hipGetLastError();
}

hipError_t launch_sweep(const SweepConfig &c_in, const void *src, void *dst, bool copy_only, hipStream_t s) {
  SweepConfig c = c_in;
  bool ext = c.solid != nullptr || c.geo_code != nullptr;
  for (int f = 0; f < 6; ++f) ext = ext || c.face_v[f] != nullptr;
  if (ext && !copy_only) {
    c.nodes_per_thread = 1;
    switch (c.storage) {
      case kStoreF64: return launch_sweep_ext<FormF64>(src, dst, make_args<double>(c), c.block_x, s);
      case kStoreF32: return launch_sweep_ext<FormF32>(src, dst, make_args<double>(c), c.block_x, s);
      case kStoreF16: return launch_sweep_ext<FormF16>(src, dst, make_args<float>(c), c.block_x, s);
      case kStoreF16SR: return launch_sweep_ext<FormF16SR>(src, dst, make_args<float>(c), c.block_x, s);
    }
    return hipErrorInvalidValue;
  }
  switch (c.storage) {
    case kStoreF64: {
      const auto a = make_args<double>(c);
      return copy_only ? launch_sweep_shape<FormF64, true>(src, dst, a, c.block_x, c.nodes_per_thread, s)
                       : launch_sweep_shape<FormF64, false>(src, dst, a, c.block_x, c.nodes_per_thread, s);
    }
    case kStoreF32: {
      const auto a = make_args<double>(c);
      return copy_only ? launch_sweep_shape<FormF32, true>(src, dst, a, c.block_x, c.nodes_per_thread, s)
                       : launch_sweep_shape<FormF32, false>(src, dst, a, c.block_x, c.nodes_per_thread, s);
    }
    case kStoreF16:
    case kStoreF16SR: {
      const auto a = make_args<float>(c);
      if (copy_only) return launch_sweep_shape<FormF16, true>(src, dst, a, c.block_x, c.nodes_per_thread, s);
      return c.storage == kStoreF16 ? launch_sweep_shape<FormF16, false>(src, dst, a, c.block_x, c.nodes_per_thread, s)
                                    : launch_sweep_shape<FormF16SR, false>(src, dst, a, c.block_x,
                                                                           c.nodes_per_thread, s);
    }
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Complex geometry (Sec. V): a wall node's rule follows from which of its
// populations stream in from solid-interior nodes (unknown).  A plane with
// inward normal n is a wall of the node when all five populations with
// c.n > 0 are unknown.  Unknown set = union of 1, 2 or 3 walls on distinct
// axes: plane, concave edge, corner (the box rules, walls at rest); a single
// unknown diagonal: convex edge; anything else: the general rule.
// ---------------------------------------------------------------------------
void classify_geometry(int nx, int ny, int nz, const unsigned char *cell, unsigned *code, long long *counts) {
  if (counts)
    for (int i = 0; i < 5; ++i) counts[i] = 0;
  unsigned plane_set[6];
  for (int f = 0; f < 6; ++f) plane_set[f] = unknown_mask(f) & 0x3ffffu;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t n = size_t(x) + size_t(nx) * (size_t(y) + size_t(ny) * size_t(z));
        unsigned c = geo_code(kGeoFluid, 0u, 0u);
        if (cell[n] == 2) {
          c = geo_code(kGeoSolid, 0u, 0u);
        } else if (cell[n] == 1) {
          unsigned U = 0;
          for (int k = 0; k < 18; ++k) {
            const int sx = (x - cx(k) + nx) % nx, sy = (y - cy(k) + ny) % ny, sz = (z - cz(k) + nz) % nz;
            if (cell[size_t(sx) + size_t(nx) * (size_t(sy) + size_t(ny) * size_t(sz))] == 2) U |= 1u << k;
          }
          unsigned m = 0, covered = 0;
          int walls = 0, axes_used = 0;
          bool distinct = true;
          for (int f = 0; f < 6; ++f)
            if ((U & plane_set[f]) == plane_set[f]) {
              m |= 1u << f;
              covered |= plane_set[f];
              ++walls;
              if (axes_used & (1 << (f / 2))) distinct = false;
              axes_used |= 1 << (f / 2);
            }
          const int nunk = __builtin_popcount(U);
          if (U == 0u)
            c = geo_code(kGeoFluid, 0u, 0u);
          else if (covered == U && walls >= 1 && walls <= 3 && distinct)
            c = geo_code(kGeoPlaneEdgeCorner, m, U);
          else if (walls == 0 && nunk == 1 && (U & 0x3ffc0u))
            c = geo_code(kGeoConvexEdge, 0u, U);
          else
            c = geo_code(kGeoGeneral, 0u, U);
        }
        code[n] = c;
        if (counts) ++counts[c >> 24];
      }
}

static unsigned blocks_for(size_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

hipError_t launch_init(int storage, void *f, size_t N, PopLayout lay, double rho0, const double u0[3],
                       hipStream_t s) {
  const dim3 g(blocks_for(N, 256)), b(256);
  switch (storage) {
    case kStoreF64: init_kernel<double><<<g, b, 0, s>>>(static_cast<double *>(f), N, lay, rho0, u0[0], u0[1], u0[2]); break;
    case kStoreF32: init_kernel<float><<<g, b, 0, s>>>(static_cast<float *>(f), N, lay, rho0, u0[0], u0[1], u0[2]); break;
    case kStoreF16:
    case kStoreF16SR: init_kernel<_Float16><<<g, b, 0, s>>>(static_cast<_Float16 *>(f), N, lay, rho0, u0[0], u0[1], u0[2]); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_moments(int storage, const void *f, PopLayout lay, size_t n0, size_t count, double *rho, double *u,
                          double *partials, int nblk, hipStream_t s) {
  const dim3 g(nblk), b(256);
  switch (storage) {
    case kStoreF64: moments_kernel<double><<<g, b, 0, s>>>(static_cast<const double *>(f), lay, n0, count, rho, u, partials); break;
    case kStoreF32: moments_kernel<float><<<g, b, 0, s>>>(static_cast<const float *>(f), lay, n0, count, rho, u, partials); break;
    case kStoreF16:
    case kStoreF16SR: moments_kernel<_Float16><<<g, b, 0, s>>>(static_cast<const _Float16 *>(f), lay, n0, count, rho, u, partials); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int nblk, double *out, hipStream_t s) {
  reduce_partials_kernel<<<dim3(1), dim3(256), 0, s>>>(partials, nblk, out);
  return hipGetLastError();
}

hipError_t launch_to_double(int storage, const void *f, PopLayout lay, size_t n0, size_t count, double *out,
                            hipStream_t s) {
  const dim3 g(blocks_for(count, 256)), b(256);
  switch (storage) {
    case kStoreF64: to_double_kernel<double><<<g, b, 0, s>>>(static_cast<const double *>(f), lay, n0, count, out); break;
    case kStoreF32: to_double_kernel<float><<<g, b, 0, s>>>(static_cast<const float *>(f), lay, n0, count, out); break;
    case kStoreF16:
    case kStoreF16SR: to_double_kernel<_Float16><<<g, b, 0, s>>>(static_cast<const _Float16 *>(f), lay, n0, count, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_from_double(int storage, void *f, PopLayout lay, size_t n0, size_t count, const double *in,
                              hipStream_t s) {
  const dim3 g(blocks_for(count, 256)), b(256);
  switch (storage) {
    case kStoreF64: from_double_kernel<double><<<g, b, 0, s>>>(static_cast<double *>(f), lay, n0, count, in); break;
    case kStoreF32: from_double_kernel<float><<<g, b, 0, s>>>(static_cast<float *>(f), lay, n0, count, in); break;
    case kStoreF16:
    case kStoreF16SR: from_double_kernel<_Float16><<<g, b, 0, s>>>(static_cast<_Float16 *>(f), lay, n0, count, in); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_relayout(int esize, const void *src, PopLayout from, void *dst, PopLayout to, size_t N,
                           hipStream_t s) {
  const dim3 g(blocks_for(N, 256)), b(256);
  switch (esize) {
    case 8: relayout_kernel<unsigned long long><<<g, b, 0, s>>>(static_cast<const unsigned long long *>(src), from,
                                                                 static_cast<unsigned long long *>(dst), to, N); break;
    case 4: relayout_kernel<unsigned><<<g, b, 0, s>>>(static_cast<const unsigned *>(src), from,
                                                       static_cast<unsigned *>(dst), to, N); break;
    case 2: relayout_kernel<unsigned short><<<g, b, 0, s>>>(static_cast<const unsigned short *>(src), from,
                                                             static_cast<unsigned short *>(dst), to, N); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void *src, void *dst, size_t nbytes, hipStream_t s) {
  const size_t n16 = nbytes / 16;
  const size_t nblk = (n16 + 255) / 256;
  if (nblk == 0) return hipSuccess;
  if (nblk > 0x7fffffffu) return hipErrorInvalidValue;
  copy_probe_kernel<<<dim3(unsigned(nblk)), dim3(256), 0, s>>>(static_cast<const uint4 *>(src),
                                                              static_cast<uint4 *>(dst), n16);
  return hipGetLastError();
}

}  // namespace lbm
