// lbm_internal.hpp -- declarations shared by the C-ABI layer and the kernel
// launchers inside the library (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/lbm.h"
#include "d3q19.hpp"
#include "node_update.hpp"

namespace lbm {

// Record a printf-style message for lbm_last_error() on this thread and
// return st.
lbm_status set_error(lbm_status st, const char *fmt, ...);

enum { kStoreF64 = 0, kStoreF32 = 1, kStoreF16 = 2, kStoreF16SR = 3 };

// Distance in elements between consecutive populations in a buffer: the
// node count rounded up to a multiple of 64, so that every population starts
// on a 128-byte cache-line boundary (for 2-, 4- and 8-byte elements) and a
// wavefront's 64 consecutive nodes touch whole lines.
inline size_t population_pitch(size_t nodes) { return (nodes + 63) / 64 * 64; }

// Where population k of node n = x + nx*r (r = y + ny*z, the x-row) lives in
// a buffer: element k*pop_stride + r*row_stride + x.  Population-major
// (structure of arrays): pop_stride = P, row_stride = nx, i.e. k*P + n.
// Row-major: pop_stride = R, row_stride = 19*R (R = row_pitch(nx) >= nx) --
// the 19 populations of one x-row lie next to each other, so a sweep streams
// through a few nearby regions instead of 19 regions P elements apart.
struct PopLayout {
  size_t pop_stride, row_stride;
  unsigned nx;
  __host__ __device__ size_t index(int k, size_t n) const {
    const size_t r = n / nx;
    return size_t(k) * pop_stride + r * row_stride + (n - r * nx);
  }
};
inline PopLayout population_major(size_t nodes, int nx) { return {population_pitch(nodes), size_t(nx), unsigned(nx)}; }

// Row pitch R of the row-major layout: nx rounded up so that every population
// row starts on a 128-byte boundary.  (A row that starts inside a cache line
// shares its first and last lines with neighbouring rows that other waves
// write: the batch sweep over lattices of arbitrary nx ran 1.8x slower.)
inline size_t row_pitch(int nx, size_t esize) {
  const size_t q = 128 / esize;
  return (size_t(nx) + q - 1) / q * q;
}
inline PopLayout row_major(int nx, size_t esize) {
  const size_t R = row_pitch(nx, esize);
  return {R, 19 * R, unsigned(nx)};
}
// Elements one population buffer needs in a layout (LBM_LAYOUT_*).
inline size_t buffer_elements(int layout, int nx, int ny, int nz, size_t esize) {
  return layout == LBM_LAYOUT_ROW_MAJOR ? 19 * row_pitch(nx, esize) * size_t(ny) * size_t(nz)
                                        : 19 * population_pitch(size_t(nx) * ny * nz);
}

// Everything one sweep launch needs, in host form.
struct SweepConfig {
  int storage;
  int nx, ny, nz;
  PopLayout layout;
  double tau;
  unsigned bc_mask;  // bit f: face f is bounded (velocity or pressure BC)
  unsigned p_mask;   // bit f: face f is a pressure face
  double v[6][3];    // face velocities (pressure faces: tangential velocity)
  double rho_p[6];   // prescribed densities of the pressure faces
  double force[3];   // body force
  unsigned rule_flags;               // kRuleNoTransverse
  const unsigned *solid;             // device [N] solid words (NodeExt), or nullptr
  const double *face_v[6];           // device per-node face velocities, or nullptr
  const unsigned *geo_code;          // device complex-geometry node codes, or nullptr
  int block_x;
  int nodes_per_thread;
  int xcd_remap;
  unsigned step;  // index of the step this launch performs (stochastic rounding)
};

// Kernel-argument form, arithmetic type T.
template <class T>
struct SweepArgs {
  int nx, ny, nz;
  size_t pop_stride, row_stride;  // PopLayout
  int nxc;                        // blocks per x-row
  unsigned nblocks;  // grid size
  int xcd_remap;
  unsigned key;  // step key of the stochastic rounding
  NodeParams<T> p;
  NodeExt ext;   // used by the extended sweep only
};

hipError_t launch_sweep(const SweepConfig &c, const void *src, void *dst, bool copy_only, hipStream_t s);
// One step (c.step) with one node per thread and block width c.block_x (64,
// 128, 256 or 512), no solid mask, face field or geometry, that also takes
// the convergence measure of the state it writes against snap ([3][N]
// floats, replaced): the wave maxima of velocity_change go to partials
// (sweep_delta_partials(c) floats, scratch), then their maximum to
// *delta_bits (zero before the call) as the bit pattern of the float.
hipError_t launch_sweep_delta(const SweepConfig &c, const void *src, void *dst, float *snap, double inv_uref,
                              float *partials, unsigned *delta_bits, hipStream_t s);
size_t sweep_delta_partials(const SweepConfig &c);
// Two steps (c.step and c.step + 1) in one pass, row-major layout, no solid
// mask, face field or geometry; z ranges of zc planes per workgroup; tiles of
// `rows` interior rows (5, or 0 for the form's default).
hipError_t launch_sweep2(const SweepConfig &c, int zc, int rows, const void *src, void *dst, hipStream_t s);

// Node codes of a complex geometry from node types (0 fluid, 1 wall node,
// 2 solid interior), all axes periodic; code[n] as geo_code().  Returns the
// number of nodes of each kind in counts[5] (fluid, solid, plane/edge/corner,
// convex edge, general) if counts is non-null.
void classify_geometry(int nx, int ny, int nz, const unsigned char *cell, unsigned *code, long long *counts);
hipError_t launch_init(int storage, void *f, size_t N, PopLayout lay, double rho0, const double u0[3],
                       hipStream_t s);
hipError_t launch_moments(int storage, const void *f, PopLayout lay, size_t n0, size_t count, double *rho, double *u,
                          double *partials, int nblk, hipStream_t s);
hipError_t launch_reduce(const double *partials, int nblk, double *out, hipStream_t s);
hipError_t launch_to_double(int storage, const void *f, PopLayout lay, size_t n0, size_t count, double *out,
                            hipStream_t s);
hipError_t launch_from_double(int storage, void *f, PopLayout lay, size_t n0, size_t count, const double *in,
                              hipStream_t s);
hipError_t launch_relayout(int esize, const void *src, PopLayout from, void *dst, PopLayout to, size_t N,
                           hipStream_t s);
hipError_t launch_copy_probe(const void *src, void *dst, size_t nbytes, hipStream_t s);

}  // namespace lbm
